"""The paper's manufactured-solution test of the field solver (Sec. "Field
solver", Eqs. r, z and mms): the meridian half plane of a spherical shell,
r_1 = 1 <= rho <= r_2 = 10, in cylindrical (r, z) coordinates, with the
geometric factor Omega = r, and the potential
phi = sin((r_2 - r_1)^2 xi (1 - xi)) cos(pi eta^2).

Its right side is the axisymmetric spherical Laplacian of phi written out in
(rho, theta) and differentiated by hand, multiplied by Omega J and the logical
cell volume (the cell-integrated form of Eq. poiscurv at the cell centre).
Boundary values: phi = 0 on xi = 0, 1 (Dirichlet), d phi / d eta = 0 on
eta = 0, 1 (the symmetry axis, Neumann).  Shared by the oracle's pins and the
GPU solver tests; it holds none of the solver's arithmetic."""
import numpy as np

import oracle as O

R1, R2 = 1.0, 10.0


def cell_centres(n):
    d = len(n)
    axes = [(np.arange(n[a]) + 0.5) / n[a] for a in range(d)]
    G = np.meshgrid(*axes, indexing="ij")
    # linear index i + n0 (j + n1 k): flatten in Fortran order
    xi = np.zeros((int(np.prod(n)), 3))
    for a in range(d):
        xi[:, a] = G[a].ravel(order="F")
    return xi


def spherical_mms(n0, n1=None):
    """(oracle map, oracle grid, exact phi at cell centres, charge per cell)."""
    n1 = n0 if n1 is None else n1
    D = R2 - R1
    A = D * D
    m = O.make_map(O.SPHERICAL_RZ, 2, r_in=R1, r_out=R2, omega=1)
    g = O.make_grid((n0, n1), bc_lo=(O.DIRICHLET, O.NEUMANN), bc_hi=(O.DIRICHLET, O.NEUMANN))
    xi = cell_centres((n0, n1))
    x, _, _, J = O.map_eval(m, xi)
    u, v = xi[:, 0], xi[:, 1]
    arg = A * u * (1 - u)
    ce = np.cos(np.pi * v ** 2)
    se = np.sin(np.pi * v ** 2)
    phi = np.sin(arg) * ce
    p_u = A * (1 - 2 * u) * np.cos(arg) * ce
    p_uu = (-2 * A * np.cos(arg) - A * A * (1 - 2 * u) ** 2 * np.sin(arg)) * ce
    p_v = -np.sin(arg) * se * 2 * np.pi * v
    p_vv = -np.sin(arg) * (ce * (2 * np.pi * v) ** 2 + se * 2 * np.pi)
    rho_s = R1 + D * u
    th = np.pi * (1 - v)
    # spherical Laplacian of phi(rho, theta), axisymmetric
    p_r = p_u / D
    p_rr = p_uu / D ** 2
    p_t = -p_v / np.pi
    p_tt = p_vv / np.pi ** 2
    lap = p_rr + 2 * p_r / rho_s + (p_tt + np.cos(th) / np.sin(th) * p_t) / rho_s ** 2
    Om = x[:, 0]
    charge = -lap * Om * J / (n0 * n1)
    return m, g, phi, charge
