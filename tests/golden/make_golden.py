"""Write oracle-computed expected energies to tests/golden/*.json.

Calls only oracle/ (CPU FP64, full occupation-basis sparse H, textbook
Lanczos, Sturm bisection) and the seeded input generators.  Each value is
the lowest Ritz value once it has changed by at most 1e-14 over three steps
in a row.

Usage:
  python tests/golden/make_golden.py [name ...]
    names: heisenberg16 hubbard12 hubbard16 j1j2_6x5 hubbard14_spatial serving
  --rows   apply H row by row (no stored matrix) instead of through CSR;
           the 6x5 J1-J2 sector's CSR takes about 86 GB of host memory, so
           it defaults to row-by-row when the host has less than 120 GB.

`serving` writes serving_2026_energies.json: one energy per request of
serving_requests(256, 2026), in request order.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2605_07621_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-14


def _host_bytes():
    try:
        return os.sysconf("SC_PAGE_SIZE") * os.sysconf("SC_PHYS_PAGES")
    except (ValueError, OSError):
        return 0


def solve(p, seed, max_steps, use_csr, log=None):
    """Oracle ground energy of problem p from the canonical start vector
    psi(seed); returns a dict of energy, steps and timings."""
    t0 = time.time()
    s = O.Sector(p.model, p.n_up, p.n_dn)
    if use_csr:
        s.csr()
    t1 = time.time()
    if log:
        log(f"  basis {s.n}, {'CSR' if use_csr else 'rows'} ready in {t1 - t0:.1f} s")
    e, a, b = s.lanczos(I.psi(seed, s.n), max_steps, tol=TOL, use_csr=use_csr)
    t2 = time.time()
    stable = len(e) >= 4 and np.all(np.abs(np.diff(e[-4:])) <= TOL)
    return {"energy": float(e[-1]), "steps": int(len(e)), "dim": int(s.n),
            "energy_change_last_step": float(abs(e[-1] - e[-2])) if len(e) > 1 else None,
            "stable_three_steps": bool(stable),
            "build_s": round(t1 - t0, 1), "lanczos_s": round(t2 - t1, 1)}


def run(name, max_steps=600, rows=False):
    p = I.WORKLOADS[name]()
    use_csr = not rows
    if name == "j1j2_6x5" and _host_bytes() < 120 * 2**30:
        use_csr = False
    print(f"[golden] {name}: start ({'CSR' if use_csr else 'rows'}, {O.num_threads()} threads)", flush=True)
    O.set_progress(5)
    r = solve(p, p.meta["seed"] + 1, max_steps, use_csr, log=lambda m: print(m, flush=True))
    out = {"workload": name, "model": p.model.name, "n_up": p.n_up, "n_dn": p.n_dn, **r,
           "tol": TOL,
           "method": ("oracle: " + ("CSR of the full occupation-basis H" if use_csr else
                                    "rows of the full occupation-basis H generated on the fly")
                      + ", 3-term Lanczos, Sturm bisection"),
           "oracle_threads": O.num_threads()}
    with open(os.path.join(HERE, f"{name}_energy.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def run_serving(n_requests=256, seed=2026):
    reqs = I.serving_requests(n_requests, seed)
    out = []
    t0 = time.time()
    for k, p in enumerate(reqs):
        r = solve(p, p.meta["seed"], 800, True)
        out.append({"k": k, "family": p.meta["family"], "n": p.meta["n"],
                    "param": p.meta.get("delta", p.meta.get("U")), **r})
        print(f"[golden] serving {k}: {p.model.name} dim {r['dim']} E={r['energy']:.15f} "
              f"steps {r['steps']} ({time.time() - t0:.0f} s)", flush=True)
    doc = {"requests": n_requests, "seed": seed, "tol": TOL,
           "method": "oracle: CSR of the full occupation-basis H, 3-term Lanczos from psi(request seed), "
                     "Sturm bisection",
           "oracle_threads": O.num_threads(), "energies": out}
    with open(os.path.join(HERE, f"serving_{seed}_energies.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    rows = "--rows" in sys.argv
    names = args or ["heisenberg16", "hubbard12", "hubbard16"]
    for n in names:
        if n == "serving":
            run_serving()
        else:
            run(n, 600, rows)
