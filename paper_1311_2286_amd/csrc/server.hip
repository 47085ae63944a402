// server.hip -- request loop over independent simulation cases (the serving
// side of the library): FIFO admission by slot and HBM budget, resident cases
// advanced one step per pump iteration (cases of one grid shape together, their
// field phases batched, on a shared stream; the others on per-slot streams), results and
// per-step latencies collected when a case finishes.  Host code on top of the
// public C ABI (cpic.h) and the HIP runtime.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "cpic.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest rank
  size_t k = (size_t)(q / 100.0 * (double)v.size() + 0.5);
  if (k < 1) k = 1;
  if (k > v.size()) k = v.size();
  return v[k - 1];
}

struct Case {
  uint64_t ticket = 0;
  cpic_case_desc desc;
  std::vector<std::vector<unsigned char>> cell, off, vel;  // host copies per species
  std::vector<double> vertices;                             // host copy of a tabulated map
  cpic_sim* sim = nullptr;
  hipStream_t stream = nullptr;
  int stream_index = -1;
  uint64_t group = 0;      // batch signature (0: the case steps alone)
  int slot = -1;
  int steps_enqueued = 0;
  hipEvent_t done_ev = nullptr;
  bool finishing = false;
  double t_submit = 0, t_admit = 0;
  long long particles0 = 0;
  cpic_case_result result;
  bool done = false;
};

}  // namespace

struct cpic_server {
  size_t budget = 0, used = 0, peak = 0;
  int max_slots = 1;
  cpic_allocator user;
  bool has_user = false;
  std::unordered_map<void*, size_t> sizes;
  std::vector<hipStream_t> streams;  // one per slot, or the caller's stream
  bool own_streams = false;
  std::vector<int> slot_busy;
  std::deque<Case*> queue;
  std::vector<Case*> active;
  std::unordered_map<uint64_t, Case*> cases;
  uint64_t next_ticket = 1;
  bool blocked = false;  // the head of the queue did not fit: wait for a case to finish
  long long submitted = 0, completed = 0, failed = 0, pushes = 0, peak_active = 0;
  std::vector<double> step_samples;
  cpic_allocator counting;  // handed to every case
  bool no_graphs = false;   // cases step without recorded graphs (CPIC_SERVER_NO_GRAPHS set)
  bool no_batch = false;    // cases step one by one (CPIC_SERVER_NO_BATCH set)
  std::vector<int> stream_load;  // active cases per stream
  // batch groups: signature -> (stream index, active cases); cases of a group share a stream
  std::unordered_map<uint64_t, std::pair<int, int>> groups;
  hipStream_t admit_stream = nullptr;  // new cases are set up here, then join their stream
  long long batched_steps = 0;   // case steps taken inside batches
};

namespace {

void* budget_alloc(size_t bytes, void* ctx) {
  cpic_server* s = (cpic_server*)ctx;
  if (s->used + bytes > s->budget) return nullptr;
  void* p = nullptr;
  if (s->has_user) {
    p = s->user.alloc(bytes, s->user.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (!p) return nullptr;
  s->sizes[p] = bytes;
  s->used += bytes;
  s->peak = std::max(s->peak, s->used);
  return p;
}

void budget_free(void* p, void* ctx) {
  cpic_server* s = (cpic_server*)ctx;
  auto it = s->sizes.find(p);
  if (it == s->sizes.end()) return;
  s->used -= it->second;
  s->sizes.erase(it);
  if (s->has_user)
    s->user.free(p, s->user.ctx);
  else
    (void)hipFree(p);
}

size_t real_bytes(const cpic_grid_desc& g) { return g.precision == CPIC_FP64 ? 8 : 4; }

// The stream of a new case: its group's, else the least loaded one.
int pick_stream(cpic_server* s, uint64_t key) {
  if (key) {
    auto it = s->groups.find(key);
    if (it != s->groups.end()) return it->second.first;
  }
  int best = 0;
  for (int i = 1; i < (int)s->stream_load.size(); ++i)
    if (s->stream_load[i] < s->stream_load[best]) best = i;
  return best;
}

void leave_stream(cpic_server* s, Case* c) {
  if (c->stream_index < 0) return;
  --s->stream_load[c->stream_index];
  if (c->group) {
    auto it = s->groups.find(c->group);
    if (it != s->groups.end() && --it->second.second == 0) s->groups.erase(it);
  }
  c->stream_index = -1;
}

void fail_case(cpic_server* s, Case* c, int status) {
  c->result.status = status;
  c->done = true;
  ++s->failed;
}

// Create the case's simulation; CPIC_E_NOMEM means it did not fit (yet).
int admit_one(cpic_server* s, Case* c, int slot) {
  const cpic_case_desc& d = c->desc;
  cpic_sim* sim = nullptr;
  hipStream_t st0 = s->admit_stream ? s->admit_stream : s->streams[0];
  int rc = cpic_create(&d.map, &d.grid, &s->counting, (void*)st0, &sim);
  if (rc != CPIC_OK) return rc;
  for (int k = 0; k < d.nspecies && rc == CPIC_OK; ++k) {
    cpic_species_desc sd = d.species[k];
    if (sd.capacity == 0) sd.capacity = std::max<size_t>(d.count[k], 1);
    int sid = -1;
    rc = cpic_add_species(sim, &sd, &sid);
    if (rc == CPIC_OK)
      rc = cpic_set_particles(sim, sid, d.count[k], (const int32_t*)c->cell[k].data(), c->off[k].data(),
                              c->vel[k].data(), nullptr, 0);
  }
  if (rc == CPIC_OK) rc = cpic_initialize(sim);
  if (rc == CPIC_OK) rc = cpic_set_timing(sim, 1);
  // one host launch per step: the loop over many small cases is host-bound otherwise
  if (rc == CPIC_OK && !s->no_graphs) rc = cpic_set_graphs(sim, 1);
  // the stream: its batch group's, else the least loaded one
  uint64_t key = 0;
  if (rc == CPIC_OK && !s->no_batch) rc = cpic_batch_signature(sim, &key);
  const int si = pick_stream(s, key);
  if (rc == CPIC_OK && s->streams[si] != st0) rc = cpic_set_stream(sim, (void*)s->streams[si]);
  if (rc != CPIC_OK) {
    cpic_destroy(sim);
    return rc;
  }
  c->sim = sim;
  c->slot = slot;
  c->stream = s->streams[si];
  c->stream_index = si;
  ++s->stream_load[si];
  c->group = key;
  if (key) {
    auto& g = s->groups[key];
    if (g.second == 0) g.first = si;
    ++g.second;
  }
  c->t_admit = now_ms();
  c->result.queue_ms = c->t_admit - c->t_submit;
  return CPIC_OK;
}

void admit(cpic_server* s) {
  while (!s->queue.empty() && !s->blocked && (int)s->active.size() < s->max_slots) {
    Case* c = s->queue.front();
    int slot = 0;
    while (s->slot_busy[slot]) ++slot;
    int rc = admit_one(s, c, slot);
    if (rc == CPIC_E_NOMEM) {
      if (s->active.empty()) {
        // nothing else holds memory: this case can never fit
        s->queue.pop_front();
        fail_case(s, c, CPIC_E_BUDGET);
        continue;
      }
      s->blocked = true;
      return;
    }
    s->queue.pop_front();
    if (rc != CPIC_OK) {
      fail_case(s, c, rc);
      continue;
    }
    s->slot_busy[slot] = 1;
    s->active.push_back(c);
    s->peak_active = std::max(s->peak_active, (long long)s->active.size());
  }
}

// Collect the result of a case whose last step has completed and free it.
void retire(cpic_server* s, Case* c) {
  cpic_case_result& r = c->result;
  cpic_diag dg;
  int rc = cpic_get_diag(c->sim, &dg);
  if (rc == CPIC_OK) {
    r.steps = (int)dg.step;
    r.kinetic = dg.kinetic;
    r.field_energy = dg.field_energy;
    r.mg_relres = dg.mg_relres;
    r.nspecies = dg.nspecies;
    for (int k = 0; k < dg.nspecies && k < CPIC_MAX_SPECIES; ++k) {
      r.count[k] = dg.count[k];
      r.absorbed[k] = dg.absorbed[k];
      r.outflow[k] = dg.outflow[k];
      r.injected[k] = dg.injected[k];
      r.qsum_lo[k] = dg.qsum_lo[k];
      r.qsum_hi[k] = dg.qsum_hi[k];
    }
    const int n = c->desc.nsteps;
    std::vector<double> st((size_t)n);
    int samples = 0;
    rc = cpic_get_timing(c->sim, n, nullptr, nullptr, nullptr, st.data(), &samples);
    if (rc == CPIC_OK) {
      st.resize((size_t)std::min(samples, n));
      r.step_p50_ms = percentile(st, 50.0);
      r.step_p99_ms = percentile(st, 99.0);
      s->step_samples.insert(s->step_samples.end(), st.begin(), st.end());
    }
  }
  if (rc == CPIC_OK && c->desc.phi_out) {
    size_t nb = cpic_field_bytes(c->sim, CPIC_FIELD_PHI);
    rc = cpic_get_field(c->sim, CPIC_FIELD_PHI, 0, c->desc.phi_out, nb, 0);
  }
  r.pushes = c->particles0 * (long long)c->desc.nsteps;
  r.service_ms = now_ms() - c->t_admit;
  r.status = rc;
  cpic_destroy(c->sim);
  c->sim = nullptr;
  (void)hipEventDestroy(c->done_ev);
  c->done_ev = nullptr;
  s->slot_busy[c->slot] = 0;
  leave_stream(s, c);
  c->done = true;
  // release the host copies of the initial particles
  c->cell.clear();
  c->off.clear();
  c->vel.clear();
  if (rc == CPIC_OK) {
    ++s->completed;
    s->pushes += r.pushes;
  } else {
    ++s->failed;
  }
  s->blocked = false;  // memory was returned: the queue head may fit now
}

}  // namespace

extern "C" cpic_status cpic_server_create(size_t hbm_budget_bytes, int max_slots, const cpic_allocator* alloc,
                                          void* hip_stream, cpic_server** out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || max_slots > 64) return CPIC_E_ARG;
  *out = nullptr;
  cpic_server* s = new cpic_server();
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  if (alloc && alloc->alloc && alloc->free) {
    s->user = *alloc;
    s->has_user = true;
  }
  s->counting.alloc = budget_alloc;
  s->counting.free = budget_free;
  s->counting.ctx = s;
  if (hip_stream) {
    s->streams.push_back((hipStream_t)hip_stream);
  } else {
    s->own_streams = true;
    if (hipStreamCreateWithFlags(&s->admit_stream, hipStreamNonBlocking) != hipSuccess) {
      s->admit_stream = nullptr;
      cpic_server_destroy(s);
      return CPIC_E_HIP;
    }
    for (int i = 0; i < max_slots; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        cpic_server_destroy(s);
        return CPIC_E_HIP;
      }
      s->streams.push_back(st);
    }
  }
  s->slot_busy.assign((size_t)max_slots, 0);
  s->stream_load.assign(s->streams.size(), 0);
  s->no_graphs = getenv("CPIC_SERVER_NO_GRAPHS") != nullptr;
  s->no_batch = getenv("CPIC_SERVER_NO_BATCH") != nullptr;
  *out = s;
  return CPIC_OK;
}

extern "C" cpic_status cpic_server_submit(cpic_server* s, const cpic_case_desc* d, uint64_t* ticket) {
  if (!s || !d || !ticket) return CPIC_E_ARG;
  if (d->nspecies < 1 || d->nspecies > CPIC_MAX_SPECIES || d->nsteps < 1) return CPIC_E_ARG;
  const int dim = d->map.dim;
  if (dim != 2 && dim != 3) return CPIC_E_ARG;
  const size_t r = real_bytes(d->grid);
  Case* c = new Case();
  c->desc = *d;
  if (d->map.kind == CPIC_MAP_TABULATED) {
    if (!d->map.vertices) {
      delete c;
      return CPIC_E_ARG;
    }
    size_t nv = 1;
    for (int a = 0; a < dim; ++a) {
      const int n = d->grid.n[a];
      if (n < 1) {
        delete c;
        return CPIC_E_ARG;
      }
      nv *= (size_t)(d->grid.bc_lo[a] == CPIC_BC_PERIODIC ? n : n + 1);
    }
    c->vertices.assign(d->map.vertices, d->map.vertices + (size_t)dim * nv);
    c->desc.map.vertices = c->vertices.data();
  }
  c->cell.resize((size_t)d->nspecies);
  c->off.resize((size_t)d->nspecies);
  c->vel.resize((size_t)d->nspecies);
  for (int k = 0; k < d->nspecies; ++k) {
    const size_t n = d->count[k];
    if (n > 0 && (!d->cell[k] || !d->off[k] || !d->vel[k])) {
      delete c;
      return CPIC_E_ARG;
    }
    c->cell[k].resize(std::max<size_t>(n, 1) * 4);
    c->off[k].resize(std::max<size_t>(n, 1) * dim * r);
    c->vel[k].resize(std::max<size_t>(n, 1) * 3 * r);
    if (n > 0) {
      memcpy(c->cell[k].data(), d->cell[k], n * 4);
      memcpy(c->off[k].data(), d->off[k], n * dim * r);
      memcpy(c->vel[k].data(), d->vel[k], n * 3 * r);
    }
    c->desc.cell[k] = nullptr;
    c->desc.off[k] = nullptr;
    c->desc.vel[k] = nullptr;
    c->particles0 += (long long)n;
  }
  memset(&c->result, 0, sizeof(c->result));
  c->result.status = CPIC_E_PENDING;
  c->ticket = s->next_ticket++;
  c->t_submit = now_ms();
  s->queue.push_back(c);
  s->cases[c->ticket] = c;
  ++s->submitted;
  *ticket = c->ticket;
  return CPIC_OK;
}

extern "C" cpic_status cpic_server_pump(cpic_server* s, int max_iterations) {
  if (!s || max_iterations < 0) return CPIC_E_ARG;
  for (int it = 0; it < max_iterations; ++it) {
    admit(s);
    if (s->active.empty()) break;
    // one step of the running cases: the cases of a batch group together
    // (their field phases batched), the others each on its own; units whose
    // step would wait for the device (cpic_step_ready) are left for the next
    // iteration while others can be stepped, so that the host keeps queueing
    // work instead of blocking on one stream
    std::map<uint64_t, std::vector<Case*>> batches;
    std::vector<std::vector<Case*>> units;
    for (Case* c : s->active) {
      if (c->finishing) continue;
      if (!c->group)
        units.push_back({c});
      else
        batches[c->group].push_back(c);
    }
    for (auto& kv : batches) units.push_back(std::move(kv.second));
    std::vector<char> go(units.size(), 0);
    bool any = false;
    for (size_t u = 0; u < units.size(); ++u) {
      int ok = 1;
      for (Case* c : units[u]) {
        int r = 1;
        if (cpic_step_ready(c->sim, &r) != CPIC_OK) r = 1;  // the step reports the error
        ok &= r;
      }
      go[u] = (char)ok;
      any |= ok != 0;
    }
    if (!any) std::fill(go.begin(), go.end(), (char)1);
    std::vector<std::pair<Case*, int>> stepped;
    for (size_t u = 0; u < units.size(); ++u) {
      if (!go[u]) continue;
      std::vector<Case*>& cs = units[u];
      if (cs.size() == 1) {
        stepped.push_back({cs[0], (int)cpic_step(cs[0]->sim, 1)});
        continue;
      }
      std::vector<cpic_sim*> sims;
      for (Case* c : cs) sims.push_back(c->sim);
      std::vector<cpic_status> st(cs.size(), CPIC_OK);
      (void)cpic_step_batch(sims.data(), (int)sims.size(), st.data());
      for (size_t i = 0; i < cs.size(); ++i) stepped.push_back({cs[i], (int)st[i]});
      s->batched_steps += (long long)cs.size();
    }
    for (auto& cr : stepped) {
      Case* c = cr.first;
      const int rc = cr.second;
      if (rc != CPIC_OK) {
        c->result.status = rc;
        c->finishing = true;
        continue;
      }
      if (++c->steps_enqueued == c->desc.nsteps) {
        c->finishing = true;
        if (hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(c->done_ev, c->stream) != hipSuccess)
          c->result.status = CPIC_E_HIP;
      }
    }
    // retire the cases whose last step has completed on the device
    std::vector<Case*> still;
    for (Case* c : s->active) {
      bool ready = false;
      if (c->finishing) {
        if (c->result.status != CPIC_E_PENDING && c->result.status != CPIC_OK) {
          ready = true;  // a failed step: retire at once
        } else {
          hipError_t q = hipEventQuery(c->done_ev);
          ready = q != hipErrorNotReady;
        }
      }
      if (ready) {
        if (c->result.status != CPIC_E_PENDING && c->result.status != CPIC_OK) {
          int status = c->result.status;
          cpic_destroy(c->sim);
          c->sim = nullptr;
          if (c->done_ev) (void)hipEventDestroy(c->done_ev);
          s->slot_busy[c->slot] = 0;
          leave_stream(s, c);
          s->blocked = false;
          fail_case(s, c, status);
        } else {
          retire(s, c);
        }
      } else {
        still.push_back(c);
      }
    }
    s->active.swap(still);
  }
  return (s->queue.empty() && s->active.empty()) ? CPIC_OK : CPIC_E_PENDING;
}

extern "C" cpic_status cpic_server_poll(cpic_server* s, uint64_t ticket, cpic_case_result* out) {
  if (!s || !out) return CPIC_E_ARG;
  auto it = s->cases.find(ticket);
  if (it == s->cases.end()) return CPIC_E_ARG;
  if (!it->second->done) return CPIC_E_PENDING;
  *out = it->second->result;
  return CPIC_OK;
}

extern "C" cpic_status cpic_server_get_stats(cpic_server* s, cpic_server_stats* out) {
  if (!s || !out) return CPIC_E_ARG;
  memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (long long)s->queue.size();
  out->active = (long long)s->active.size();
  out->peak_active = s->peak_active;
  out->budget_bytes = s->budget;
  out->used_bytes = s->used;
  out->peak_bytes = s->peak;
  out->pushes = s->pushes;
  out->step_samples = (long long)s->step_samples.size();
  out->step_p50_ms = percentile(s->step_samples, 50.0);
  out->step_p99_ms = percentile(s->step_samples, 99.0);
  out->batched_steps = s->batched_steps;
  return CPIC_OK;
}

extern "C" void cpic_server_destroy(cpic_server* s) {
  if (!s) return;
  for (Case* c : s->active) {
    if (c->sim) cpic_destroy(c->sim);
    if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  }
  for (auto& kv : s->cases) delete kv.second;
  if (s->own_streams) {
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->admit_stream) (void)hipStreamDestroy(s->admit_stream);
  }
  delete s;
}
