"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This module holds model descriptions (lattices, bonds, couplings), sector
choices, cut choices and seeded random vectors.  It holds none of the
method's arithmetic (no Hamiltonian entries, no bases, no layouts), so both
the oracle side and the product side may import it.  It imports numpy only.

Workloads follow the model benchmarks of the paper (spin-1/2 Heisenberg and
Hubbard chains, a 2d spin lattice with a spatial cut, and the spin-group
"up/down" cut of Fig. 1(c)); sizes are the ones this project measures.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Model:
    kind: str                      # "spin" | "hubbard"
    n_sites: int
    bonds: np.ndarray              # (n_bonds, 2) int32 site pairs
    jxy: Optional[np.ndarray] = None   # spin: coupling of Sx Sx + Sy Sy per bond
    jz: Optional[np.ndarray] = None    # spin: coupling of Sz Sz per bond
    t: Optional[np.ndarray] = None     # Hubbard: hopping per bond, term -t (c+c + h.c.)
    u: Optional[np.ndarray] = None     # Hubbard: on-site U per site
    name: str = ""
    v: Optional[np.ndarray] = None     # Hubbard: density interaction V n_i n_j per bond (n = n_up + n_dn)


@dataclass
class Cut:
    kind: str                      # "spatial" | "updn"
    left_mask: int = 0             # spatial: bit i set = site i belongs to the left part


@dataclass
class Problem:
    model: Model
    cut: Cut
    n_up: int
    n_dn: int = 0
    meta: dict = field(default_factory=dict)


def _arr(x, n):
    return np.full(n, float(x)) if np.isscalar(x) else np.asarray(x, dtype=np.float64)


def xxz_chain(n, J=1.0, delta=1.0, periodic=False, name=""):
    bonds = [(i, i + 1) for i in range(n - 1)] + ([(n - 1, 0)] if periodic and n > 2 else [])
    b = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    return Model("spin", n, b, jxy=_arr(J, len(b)), jz=_arr(J * delta, len(b)),
                 name=name or f"xxz_chain_{n}")


def heisenberg_chain(n, J=1.0, periodic=False):
    return xxz_chain(n, J, 1.0, periodic, name=f"heisenberg_chain_{n}")


def j1j2_lattice(lx, ly, J1=1.0, J2=0.5):
    """Open lx x ly square lattice, site index = ly*x + y.  J1 on nearest
    neighbours, J2 on both diagonals of every plaquette."""
    def s(x, y):
        return ly * x + y
    bonds, J = [], []
    for x in range(lx):
        for y in range(ly):
            if x + 1 < lx:
                bonds.append((s(x, y), s(x + 1, y))); J.append(J1)
            if y + 1 < ly:
                bonds.append((s(x, y), s(x, y + 1))); J.append(J1)
    for x in range(lx - 1):
        for y in range(ly - 1):
            bonds.append((s(x, y), s(x + 1, y + 1))); J.append(J2)
            bonds.append((s(x + 1, y), s(x, y + 1))); J.append(J2)
    b = np.asarray(bonds, dtype=np.int32)
    J = np.asarray(J)
    return Model("spin", lx * ly, b, jxy=J.copy(), jz=J.copy(), name=f"j1j2_{lx}x{ly}")


def hubbard_chain(n, t=1.0, U=4.0, periodic=False, V=None):
    """Hubbard chain; V (optional) adds V n_i n_{i+1} on every bond (the
    extended model of the paper's spatial-cut benchmark)."""
    bonds = [(i, i + 1) for i in range(n - 1)] + ([(n - 1, 0)] if periodic and n > 2 else [])
    b = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    return Model("hubbard", n, b, t=_arr(t, len(b)), u=_arr(U, n), name=f"hubbard_chain_{n}",
                 v=None if V is None else _arr(V, len(b)))


def random_spin_model(rng, n, n_bonds=None):
    """Random couplings on random distinct bonds (tiny parity cases)."""
    n_bonds = min(n_bonds or max(1, (3 * n) // 2), n * (n - 1) // 2)
    pairs = set()
    while len(pairs) < n_bonds:
        i, j = rng.integers(0, n, 2)
        if i != j:
            pairs.add((int(min(i, j)), int(max(i, j))))
    b = np.asarray(sorted(pairs), dtype=np.int32)
    return Model("spin", n, b, jxy=rng.uniform(-1, 1.5, len(b)), jz=rng.uniform(-1, 1.5, len(b)),
                 name=f"random_spin_{n}")


def random_hubbard_model(rng, n, n_bonds=None):
    """Random hoppings on random (also long-range) bonds, random U_i."""
    n_bonds = min(n_bonds or max(1, (3 * n) // 2), n * (n - 1) // 2)
    pairs = set()
    while len(pairs) < n_bonds:
        i, j = rng.integers(0, n, 2)
        if i != j:
            pairs.add((int(min(i, j)), int(max(i, j))))
    b = np.asarray(sorted(pairs), dtype=np.int32)
    return Model("hubbard", n, b, t=rng.uniform(-1.2, 1.2, len(b)), u=rng.uniform(0, 6, n),
                 name=f"random_hubbard_{n}")


def random_extended_hubbard_model(rng, n, n_bonds=None):
    """Random hoppings, U_i and bond interactions V_b on random bonds."""
    m = random_hubbard_model(rng, n, n_bonds)
    m.v = rng.uniform(-1.0, 2.5, len(m.bonds))
    m.name = f"random_ext_hubbard_{n}"
    return m


def left_mask_first(k):
    """Spatial cut with sites 0..k-1 on the left."""
    return (1 << k) - 1


def psi(seed, dim):
    """Seeded N(0,1) FP64 vector in canonical (integer-ordered) basis order."""
    return np.random.default_rng(seed).standard_normal(dim)


# ---- the five measured workloads ------------------------------------------

def heisenberg16():
    """Spin-1/2 Heisenberg open chain, N=16, J=1, Sz=0, cut 8|8."""
    return Problem(heisenberg_chain(16), Cut("spatial", left_mask_first(8)), 8,
                   meta=dict(seed=1001, lanczos_steps=100))


def hubbard12():
    """Hubbard open chain, 12 sites, t=1, U=4, N_up=N_dn=6, up/down cut."""
    return Problem(hubbard_chain(12, 1.0, 4.0), Cut("updn"), 6, 6,
                   meta=dict(seed=1002, lanczos_steps=200))


def hubbard16(U=8.0):
    """Hubbard open chain, 16 sites, t=1, U=8, N_up=N_dn=8, up/down cut."""
    return Problem(hubbard_chain(16, 1.0, U), Cut("updn"), 8, 8,
                   meta=dict(seed=1003, lanczos_tol=1e-10, lanczos_keep=150))


def j1j2_6x5():
    """J1-J2 Heisenberg on a 6x5 open lattice, J1=1, J2=0.5, Sz=0, cut x<=2 | x>=3."""
    m = j1j2_lattice(6, 5, 1.0, 0.5)
    return Problem(m, Cut("spatial", left_mask_first(15)), 15, meta=dict(seed=1004))


def hubbard14_spatial():
    """Extended Hubbard open chain of the paper's spatial-cut ED benchmark:
    14 sites, t=1, U=4, V=1 on every bond, N_up=N_dn=7, cut 7|7
    (11,778,624 amplitudes in 64 blocks (N_up_L, N_dn_L))."""
    return Problem(hubbard_chain(14, 1.0, 4.0, V=1.0), Cut("spatial", left_mask_first(7)), 7, 7,
                   meta=dict(seed=1005))


WORKLOADS = {
    "heisenberg16": heisenberg16,
    "hubbard12": hubbard12,
    "hubbard16": hubbard16,
    "j1j2_6x5": j1j2_6x5,
    "hubbard14_spatial": hubbard14_spatial,
}


def serving_requests(n_requests=256, seed=2026):
    """Mixed ground-state requests: half XXZ chains (N in {12..24} even,
    Delta ~ U[0.5, 2], J=1, Sz=0, cut N/2|N/2), half Hubbard chains
    (L in {8,10,12,14}, U ~ U[0,10], t=1, half filling, up/down cut).
    Each request carries its own start-vector seed."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_requests):
        if rng.random() < 0.5:
            n = int(rng.choice([12, 14, 16, 18, 20, 22, 24]))
            d = float(rng.uniform(0.5, 2.0))
            p = Problem(xxz_chain(n, 1.0, d), Cut("spatial", left_mask_first(n // 2)), n // 2,
                        meta=dict(family="xxz", n=n, delta=d))
        else:
            L = int(rng.choice([8, 10, 12, 14]))
            U = float(rng.uniform(0.0, 10.0))
            p = Problem(hubbard_chain(L, 1.0, U), Cut("updn"), L // 2, L // 2,
                        meta=dict(family="hubbard", n=L, U=U))
        p.meta["seed"] = int(rng.integers(1, 2**31 - 1))
        out.append(p)
    return out


def poisson_arrivals(n, rate, seed=2026):
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed + 17)
    return np.cumsum(rng.exponential(1.0 / rate, n))
