"""The oracle's pins are strong enough to catch plausible mistakes.

Each case compiles oracle.c with one deliberate mistake (ORC_PLANT, on the
CPU, into a temporary library) and runs the pin suite against it in a fresh
interpreter: the suite must fail.  The normal library (ORC_PLANT = 0) passes
the same suite in test_oracle_pins.py."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import build as B  # noqa: E402

PLANTS = {
    1: "on-site U term dropped",
    2: "fermion sign of hops dropped",
    3: "spin flip amplitude jxy instead of jxy/2",
    4: "Sz Sz evaluated with the first site twice",
    5: "only the down spins hop",
    6: "wrong sign of the beta term in Lanczos",
    7: "Lanczos stops after one step within tol instead of three",
    8: "c+ / c of one mode without its fermion sign",
    9: "bond density interaction V dropped",
    10: "spatial Hubbard cut without the reordering sign",
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_pins_catch_planted_mistake(tmp_path, plant):
    lib = B.build(out=str(tmp_path / f"liboracle_plant{plant}.so"), plant=plant)
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins did not catch: {PLANTS[plant]}\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout, r.stdout[-2000:]
