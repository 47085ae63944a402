"""Reader of tests/golden/paper_values.txt (values printed in the paper)."""
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def paper_value(key):
    with open(_PATH) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split(None, 2)
            if parts[0] == key:
                return float(parts[1])
    raise KeyError(key)
