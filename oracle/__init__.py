"""Python face of the CPU FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  Imported by tests/, __graft_entry__.smoke() and
the cpu_baseline leg of bench.py; the product package never imports it and it
never imports the product package (model descriptions arrive as plain
arrays from the seeded input generators).

Everything here is computed in the full occupation basis of one sector
(Eq. 1 of the paper written out term by term), not in the bipartite form.
"""
import ctypes
import os

import numpy as np

from . import build as _build

ORC_SPIN = 1
ORC_HUBBARD = 2
ORC_CUT_SPATIAL = 1
ORC_CUT_UPDN = 2

_lib = None


class _Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("n_bonds", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("bi", ctypes.c_void_p), ("bj", ctypes.c_void_p),
                ("jxy", ctypes.c_void_p), ("jz", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: another build of oracle.c (the planted-mistake test)
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        i64, i32, vp, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_sector_size.restype = i64
        L.orc_sector_size.argtypes = [ctypes.c_int] * 4
        L.orc_enumerate.restype = i64
        L.orc_enumerate.argtypes = [ctypes.c_int] * 4 + [vp]
        L.orc_enumerate_bruteforce.restype = i64
        L.orc_enumerate_bruteforce.argtypes = [ctypes.c_int, ctypes.c_int, vp]
        L.orc_find.restype = i64
        L.orc_find.argtypes = [vp, i64, ctypes.c_uint64]
        L.orc_build_csr.restype = i64
        L.orc_build_csr.argtypes = [vp, vp, i64, vp, vp, vp]
        L.orc_build_csr_rows.restype = i64
        L.orc_build_csr_rows.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp]
        L.orc_apply_cdag.restype = ctypes.c_int
        L.orc_apply_cdag.argtypes = [ctypes.c_int, vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
        L.orc_set_progress.restype = None
        L.orc_set_progress.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_spmv_csr.restype = None
        L.orc_spmv_csr.argtypes = [i64, vp, vp, vp, vp, vp]
        L.orc_apply_rows.restype = ctypes.c_int
        L.orc_apply_rows.argtypes = [vp, vp, i64, vp, vp, i64, vp]
        L.orc_apply_full.restype = ctypes.c_int
        L.orc_apply_full.argtypes = [vp, vp, i64, vp, vp]
        L.orc_bipartite_positions.restype = ctypes.c_int
        L.orc_bipartite_positions.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                              ctypes.c_int, ctypes.c_int, vp, i64, vp, vp, ctypes.c_int]
        L.orc_bipartite_hubbard_spatial.restype = ctypes.c_int
        L.orc_bipartite_hubbard_spatial.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, i64,
                                                    vp, vp, vp, ctypes.c_int]
        L.orc_tridiag_eig.restype = dbl
        L.orc_tridiag_eig.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int]
        L.orc_lanczos.restype = ctypes.c_int
        L.orc_lanczos.argtypes = [vp, vp, i64, vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, dbl,
                                  vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleModel:
    """Holds the model arrays alive and the C struct that points at them.

    `m` is any object with attributes kind ('spin'|'hubbard'), n_sites,
    bonds (k x 2 int), and jxy/jz (spin) or t/u (Hubbard)."""

    def __init__(self, m):
        self.kind = ORC_SPIN if m.kind == "spin" else ORC_HUBBARD
        self.n_sites = int(m.n_sites)
        b = np.ascontiguousarray(np.asarray(m.bonds, dtype=np.int32).reshape(-1, 2))
        self.bi = np.ascontiguousarray(b[:, 0])
        self.bj = np.ascontiguousarray(b[:, 1])
        self.n_bonds = len(self.bi)
        z = np.zeros(max(self.n_bonds, 1))
        if self.kind == ORC_SPIN:
            self.jxy = np.ascontiguousarray(m.jxy, dtype=np.float64)
            self.jz = np.ascontiguousarray(m.jz, dtype=np.float64)
            self.t, self.u = z, None
        else:
            self.t = np.ascontiguousarray(m.t, dtype=np.float64)
            self.u = None if m.u is None else np.ascontiguousarray(m.u, dtype=np.float64)
            v = getattr(m, "v", None)
            self.v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
            self.jxy = self.jz = z
        if self.kind == ORC_SPIN:
            self.v = None
        self.c = _Model(self.kind, self.n_sites, self.n_bonds, 0,
                        _ptr(self.bi), _ptr(self.bj), _ptr(self.jxy), _ptr(self.jz),
                        _ptr(self.t), _ptr(self.u), _ptr(self.v))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def num_threads():
    return lib().orc_num_threads()


def sector_size(kind, n_sites, n_up, n_dn=0):
    k = ORC_SPIN if kind == "spin" else ORC_HUBBARD
    return lib().orc_sector_size(k, n_sites, n_up, n_dn)


def enumerate_basis(kind, n_sites, n_up, n_dn=0):
    """Sector basis words in increasing integer order (uint64)."""
    k = ORC_SPIN if kind == "spin" else ORC_HUBBARD
    n = lib().orc_enumerate(k, n_sites, n_up, n_dn, None)
    if n < 0:
        raise ValueError("unsupported sector")
    w = np.empty(n, dtype=np.uint64)
    lib().orc_enumerate(k, n_sites, n_up, n_dn, _ptr(w))
    return w


def enumerate_bruteforce(n_sites, n_up):
    n = lib().orc_enumerate_bruteforce(n_sites, n_up, None)
    w = np.empty(n, dtype=np.uint64)
    lib().orc_enumerate_bruteforce(n_sites, n_up, _ptr(w))
    return w


class Sector:
    """One symmetry sector of one model in the occupation basis."""

    def __init__(self, model, n_up, n_dn=0):
        self.model = model
        self.om = OracleModel(model)
        self.n_up, self.n_dn = int(n_up), int(n_dn)
        self.words = enumerate_basis(model.kind, model.n_sites, n_up, n_dn)
        self.n = len(self.words)
        self._csr = None

    def find(self, w):
        return lib().orc_find(_ptr(self.words), self.n, int(w))

    def csr(self):
        if self._csr is None:
            rp = np.empty(self.n + 1, dtype=np.int64)
            nnz = lib().orc_build_csr(self.om.ref, _ptr(self.words), self.n, _ptr(rp), None, None)
            if nnz < 0:
                raise RuntimeError(f"oracle CSR build failed ({nnz})")
            col = np.empty(nnz, dtype=np.int32)
            val = np.empty(nnz, dtype=np.float64)
            r = lib().orc_build_csr(self.om.ref, _ptr(self.words), self.n, _ptr(rp), _ptr(col), _ptr(val))
            if r < 0:
                raise RuntimeError(f"oracle CSR fill failed ({r})")
            self._csr = (rp, col, val)
        return self._csr

    def dense(self):
        rp, col, val = self.csr()
        H = np.zeros((self.n, self.n))
        for r in range(self.n):
            H[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
        return H

    def apply(self, x, use_csr=True):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        if use_csr:
            rp, col, val = self.csr()
            lib().orc_spmv_csr(self.n, _ptr(rp), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
        else:
            if lib().orc_apply_full(self.om.ref, _ptr(self.words), self.n, _ptr(x), _ptr(y)):
                raise RuntimeError("oracle apply failed")
        return y

    def csr_rows(self, r0, r1):
        """CSR of rows [r0, r1) (row_ptr from 0; columns index the whole
        sector)."""
        rp = np.empty(r1 - r0 + 1, dtype=np.int64)
        nnz = lib().orc_build_csr_rows(self.om.ref, _ptr(self.words), self.n, r0, r1, _ptr(rp), None, None)
        if nnz < 0:
            raise RuntimeError(f"oracle CSR build failed ({nnz})")
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz, dtype=np.float64)
        if lib().orc_build_csr_rows(self.om.ref, _ptr(self.words), self.n, r0, r1, _ptr(rp), _ptr(col), _ptr(val)) < 0:
            raise RuntimeError("oracle CSR fill failed")
        return rp, col, val

    def apply_rows(self, x, rows):
        x = np.ascontiguousarray(x, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        y = np.empty(len(rows))
        if lib().orc_apply_rows(self.om.ref, _ptr(self.words), self.n, _ptr(x), _ptr(rows), len(rows), _ptr(y)):
            raise RuntimeError("oracle apply_rows failed")
        return y

    def bipartite_signed(self, left_mask):
        """Hubbard model, spatial cut: (pos, sign, blocks) with
        bip[pos[i]] = sign[i] * canon[i]; blocks = int64 rows
        (N_up_L, N_dn_L, d_L, d_R, offset) in lexicographic order."""
        pos = np.empty(self.n, dtype=np.int64)
        sign = np.empty(self.n, dtype=np.int8)
        blocks = np.empty(5 * 33 * 33, dtype=np.int64)
        nb = lib().orc_bipartite_hubbard_spatial(self.model.n_sites, int(left_mask), self.n_up, self.n_dn,
                                                 _ptr(self.words), self.n, _ptr(pos), _ptr(sign), _ptr(blocks),
                                                 33 * 33)
        if nb < 0:
            raise ValueError(f"oracle spatial Hubbard map failed ({nb})")
        return pos, sign, blocks[:5 * nb].reshape(nb, 5).copy()

    def bipartite(self, cut_kind, left_mask=0):
        """(pos, blocks): pos[i] = bipartite position of canonical index i;
        blocks = int64 array of rows (q_l, d_L, d_R, offset)."""
        ck = ORC_CUT_SPATIAL if cut_kind == "spatial" else ORC_CUT_UPDN
        pos = np.empty(self.n, dtype=np.int64)
        blocks = np.empty(4 * 65, dtype=np.int64)
        nb = lib().orc_bipartite_positions(self.om.kind, ck, self.model.n_sites, int(left_mask),
                                           self.n_up, self.n_dn, _ptr(self.words), self.n,
                                           _ptr(pos), _ptr(blocks), 65)
        if nb < 0:
            raise ValueError(f"oracle bipartite map failed ({nb})")
        return pos, blocks[:4 * nb].reshape(nb, 4).copy()

    def lanczos(self, v0, max_steps, reorth=False, tol=0.0, use_csr=True):
        """Returns (energies per step, alpha, beta)."""
        v0 = np.ascontiguousarray(v0, dtype=np.float64)
        a = np.zeros(max_steps)
        b = np.zeros(max_steps)
        e = np.zeros(max_steps)
        basis = np.empty((max_steps, self.n)) if reorth else None
        if use_csr:
            rp, col, val = self.csr()
        else:
            rp = col = val = None
        s = lib().orc_lanczos(self.om.ref, _ptr(self.words), self.n, _ptr(rp), _ptr(col), _ptr(val),
                              _ptr(v0), max_steps, 1 if reorth else 0, tol,
                              _ptr(a), _ptr(b), _ptr(e), _ptr(basis))
        if s < 0:
            raise RuntimeError(f"oracle lanczos failed ({s})")
        return e[:s].copy(), a[:s].copy(), b[:s].copy()


def set_progress(every):
    """Print every `every`-th Lanczos step's energy to stderr (0: off)."""
    lib().orc_set_progress(int(every))


def set_threads(n):
    """OpenMP threads of the oracle's loops from now on."""
    lib().orc_set_threads(int(n))


def spmv_csr(rp, col, val, x):
    """y = A x for a CSR block of rows (as returned by Sector.csr_rows)."""
    y = np.empty(len(rp) - 1)
    lib().orc_spmv_csr(len(rp) - 1, _ptr(rp), _ptr(col), _ptr(val), _ptr(np.ascontiguousarray(x)), _ptr(y))
    return y


def tridiag_eig(alpha, beta, k=0):
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if len(b) < max(len(a) - 1, 1):
        b = np.concatenate([b, np.zeros(max(len(a) - 1, 1) - len(b))])
    return lib().orc_tridiag_eig(_ptr(a), _ptr(b), len(a), k)


# ---------------------------------------------------------------- ground state, entanglement spectrum

def ground_state(sector, v0, tol=1e-14):
    """Lowest eigenpair of the sector's H (its CSR) by the implicitly
    restarted Lanczos method of ARPACK (scipy), started from v0.  Returns
    (energy, unit vector in canonical order)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    rp, col, val = sector.csr()
    A = sp.csr_matrix((val, col, rp), shape=(sector.n, sector.n))
    w, v = sla.eigsh(A, k=1, which="SA", tol=tol, v0=np.asarray(v0, dtype=np.float64))
    g = v[:, 0]
    return float(w[0]), g / np.linalg.norm(g)


def entanglement(sector, psi, cut_kind, left_mask=0, parts=None, cutoff=1e-14):
    """Entanglement spectrum of psi (canonical order) across the cut: the
    eigenvalues of rho_L = Tr_R |psi><psi| / <psi|psi> (the paper's
    H_E = -log rho_L), block by block of the oracle's own bipartite map, from
    the singular values of each block (numpy SVD).  Returns a dict: lam
    (per block, descending), w_q = sum_i lam_{q,i}, chi_q = #(lam > cutoff),
    n_eff = 1/sum (chi_q/sum chi)^2, weight_ipr = 1/sum W_q^2, entropy, and
    w_p[p] = sum_{q in part p} W_q^2 when parts (block -> part) is given."""
    psi = np.asarray(psi, dtype=np.float64)
    flat = np.empty_like(psi)
    if sector.model.kind == "hubbard" and cut_kind == "spatial":
        # fermion modes split by site: the signed map of the two parts'
        # ordered products (blocks labelled by (N_up_L, N_dn_L))
        pos, sign, b5 = sector.bipartite_signed(left_mask)
        flat[pos] = sign * psi
        blocks = b5[:, [0, 2, 3, 4]]
    else:
        pos, blocks = sector.bipartite(cut_kind, left_mask)
        flat[pos] = psi
    norm2 = float(psi @ psi)
    lam = []
    for q_l, d_l, d_r, off in blocks:
        m = flat[off:off + d_l * d_r].reshape(d_l, d_r)
        sv = np.linalg.svd(m, compute_uv=False) if m.size else np.zeros(0)
        lam.append(np.sort(sv * sv / norm2)[::-1][:min(d_l, d_r)])
    w_q = np.array([l.sum() for l in lam])
    chi = np.array([int(np.sum(l > cutoff)) for l in lam])
    c = chi / max(chi.sum(), 1)
    allv = np.concatenate(lam)
    pos_l = allv[allv > 0]
    out = dict(lam=lam, w_q=w_q, chi_q=chi, n_eff=1.0 / np.sum(c * c), weight_ipr=1.0 / np.sum(w_q * w_q),
               entropy=float(-np.sum(pos_l * np.log(pos_l))), blocks=blocks)
    if parts is not None:
        parts = np.asarray(parts)
        out["w_p"] = np.array([np.sum(w_q[parts == p] ** 2) for p in range(int(parts.max()) + 1)])
    return out


# ---------------------------------------------------------------- dynamical correlations

def apply_cdag(src, dst, site, spin, dagger, x):
    """y = c+_{site,spin} x (dagger) or c_{site,spin} x between the Hubbard
    sectors src and dst (canonical order of each)."""
    y = np.empty(dst.n)
    r = lib().orc_apply_cdag(src.model.n_sites, _ptr(src.words), src.n, _ptr(dst.words), dst.n, int(site), int(spin),
                             1 if dagger else 0, _ptr(np.ascontiguousarray(x, dtype=np.float64)), _ptr(y))
    if r:
        raise ValueError(f"oracle apply_cdag failed ({r})")
    return y


def continued_fraction(alpha, beta, weight, e0, dagger, omega, eta):
    """Green's function from Lanczos coefficients of H on the start vector
    c+ psi0 / |c+ psi0| (dagger) or c psi0 / |c psi0|:
      G+(w) = weight / (z - a0 - b0^2 / (z - a1 - b1^2 / ...)),  z = w + i eta + E0;
      G-(w) = weight / (z + a0 - b0^2 / (z + a1 - ...)),         z = w + i eta - E0;
    beta[j] joins steps j and j + 1 (the last one is not used)."""
    omega = np.asarray(omega, dtype=np.float64)
    z = omega + 1j * eta + (e0 if dagger else -e0)
    sgn = 1.0 if dagger else -1.0
    g = np.zeros_like(z)
    for j in range(len(alpha) - 1, -1, -1):
        tail = beta[j] ** 2 * g if j + 1 < len(alpha) else 0.0
        g = 1.0 / (z - sgn * alpha[j] - tail)
    return weight * g

