"""Write oracle-computed expected energies to tests/golden/*.json.

Calls only oracle/ (CPU FP64, full occupation-basis sparse H, textbook
Lanczos, Sturm bisection) and the seeded input generators.  Each value is
the lowest Ritz value after the energy has been stable to 1e-13 for three
steps.  Usage: python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2605_07621_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(name, max_steps):
    p = I.WORKLOADS[name]()
    t0 = time.time()
    s = O.Sector(p.model, p.n_up, p.n_dn)
    s.csr()
    t1 = time.time()
    e, a, b = s.lanczos(I.psi(p.meta["seed"] + 1, s.n), max_steps, tol=1e-13)
    t2 = time.time()
    out = {"workload": name, "model": p.model.name, "n_up": p.n_up, "n_dn": p.n_dn, "dim": int(s.n),
           "energy": float(e[-1]), "steps": int(len(e)), "energy_change_last_step": float(abs(e[-1] - e[-2])),
           "method": "oracle: CSR of the full occupation-basis H, 3-term Lanczos, Sturm bisection",
           "oracle_threads": O.num_threads(), "build_s": round(t1 - t0, 1), "lanczos_s": round(t2 - t1, 1)}
    with open(os.path.join(HERE, f"{name}_energy.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["heisenberg16", "hubbard12", "hubbard16"]
    for n in names:
        run(n, 600)
