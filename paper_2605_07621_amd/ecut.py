"""Python binding of libecut.so (include/ecut.h).

Argument marshalling only: every step of H*psi, the Lanczos solver and the
server runs in the library (host C++ sector builder + HIP kernels for
gfx950).  torch supplies device memory (tensor.data_ptr()) and streams.
The library is required: importing this module raises if libecut.so is
missing or fails to load, there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ECUT_LIB: another build of the same library (the host-sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("ECUT_LIB") or os.path.join(_HERE, "libecut.so")

ECUT_OK, ECUT_EINVAL, ECUT_ENOMEM, ECUT_EDEVICE, ECUT_ENOTCONV, ECUT_EUNSUPPORTED, ECUT_EAGAIN = 0, -1, -2, -3, -4, -5, -6
ECUT_SPIN_HALF, ECUT_HUBBARD = 1, 2
ECUT_CUT_SPATIAL, ECUT_CUT_UPDN = 1, 2
ECUT_BUILD_HOST_ONLY = 1

_STATUS = {0: "ECUT_OK", -1: "ECUT_EINVAL", -2: "ECUT_ENOMEM", -3: "ECUT_EDEVICE", -4: "ECUT_ENOTCONV",
           -5: "ECUT_EUNSUPPORTED", -6: "ECUT_EAGAIN"}


class EcutError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64, _dbl, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t


class ModelDesc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("n_sites", _i32), ("n_bonds", _i32), ("reserved", _i32),
                ("bond_i", _vp), ("bond_j", _vp), ("jxy", _vp), ("jz", _vp), ("t", _vp), ("u", _vp), ("v", _vp)]


class CutDesc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("reserved", _i32), ("left_mask", _u64)]


class QNum(ctypes.Structure):
    _fields_ = [("n_up", _i32), ("n_dn", _i32)]


class SectorsInfo(ctypes.Structure):
    _fields_ = [("dim", _i64), ("n_blocks", _i32), ("n_left_sites", _i32), ("n_right_sites", _i32),
                ("max_d_r", _i32), ("n_cut_bonds", _i32), ("n_cross_offdiag", _i32), ("n_cross_diag", _i32),
                ("kernel", _i32), ("kernel_flags", _i32), ("reserved", _i32), ("device_bytes", _i64),
                ("n_eff", _dbl)]


class LanczosOpts(ctypes.Structure):
    _fields_ = [("max_steps", _i32), ("max_restarts", _i32), ("reorth", _i32), ("fixed_steps", _i32), ("tol", _dbl),
                ("use_graph", _i32)]


class LanczosStats(ctypes.Structure):
    _fields_ = [("steps", _i32), ("restarts", _i32), ("converged", _i32), ("reserved", _i32),
                ("residual", _dbl), ("seconds", _dbl)]


class Tuning(ctypes.Structure):
    _fields_ = [("grid", _i32), ("n_xcd", _i32), ("row_order", _i32), ("variant", _i32), ("tile", _i32)]


def _tuning_dict(t):
    return dict(grid=t.grid, n_xcd=t.n_xcd, row_order=t.row_order, variant=t.variant, tile=t.tile)


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_active", _i32), ("max_steps", _i32), ("tol", _dbl), ("sequential", _i32), ("use_graph", _i32),
                ("autotune", _i32), ("large_dim", _i64)]


class Result(ctypes.Structure):
    _fields_ = [("req_id", _u64), ("status", _i32), ("steps", _i32), ("energy", _dbl), ("residual", _dbl),
                ("t_submit", _dbl), ("t_admit", _dbl), ("t_done", _dbl)]


# (name, restype, argtypes) of every entry point declared in include/ecut.h
# ecut_alloc_fn / ecut_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(_vp, _sz, _i32, _vp)
FREE_FN = ctypes.CFUNCTYPE(None, _vp, _sz, _i32, _vp)

class Entanglement(ctypes.Structure):
    _fields_ = [("n_blocks", _i32), ("n_parts", _i32), ("n_lambda", _i64), ("norm2", _dbl), ("weight_ipr", _dbl),
                ("n_eff", _dbl), ("entropy", _dbl)]


SYMBOLS = [
    ("ecut_build_sectors", _i32, [ctypes.POINTER(ModelDesc), ctypes.POINTER(CutDesc), QNum, _u32, ctypes.POINTER(_vp)]),
    ("ecut_sectors_free", None, [_vp]),
    ("ecut_sectors_get_info", _i32, [_vp, ctypes.POINTER(SectorsInfo)]),
    ("ecut_sectors_blocks", _i32, [_vp, _vp]),
    ("ecut_sectors_words", _i32, [_vp, _i32, _vp, _vp]),
    ("ecut_canonical_positions", _i32, [_vp, _vp]),
    ("ecut_canonical_signs", _i32, [_vp, _vp]),
    ("ecut_sectors_labels", _i32, [_vp, _vp]),
    ("ecut_import", _i32, [_vp, _vp, _vp, _vp]),
    ("ecut_export", _i32, [_vp, _vp, _vp, _vp]),
    ("ecut_apply_H", _i32, [_vp, _vp, _vp, _vp]),
    ("ecut_apply_H_batch", _i32, [_i32, _vp, _vp, _vp, _vp]),
    ("ecut_apply_H_batch_noalloc", _i32, [_i32, _vp, _vp, _vp, _vp]),
    ("ecut_get_tuning", _i32, [_vp, ctypes.POINTER(Tuning)]),
    ("ecut_set_tuning", _i32, [_vp, ctypes.POINTER(Tuning)]),
    ("ecut_autotune", _i32, [_vp, _vp, _vp, _vp, ctypes.POINTER(Tuning)]),
    ("ecut_lanczos_workspace", _sz, [_vp, ctypes.POINTER(LanczosOpts)]),
    ("ecut_lanczos_ground_state", _i32, [_vp, _vp, ctypes.POINTER(LanczosOpts), ctypes.POINTER(_dbl), _vp,
                                         ctypes.POINTER(LanczosStats), _vp, _vp]),
    ("ecut_apply_cdag", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    ("ecut_lanczos_tridiag", _i32, [_vp, _vp, _i32, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_dbl), _vp, _vp]),
    ("ecut_continued_fraction", _i32, [_vp, _vp, _i32, _dbl, _dbl, _i32, _vp, _i32, _dbl, _vp, _vp]),
    ("ecut_entanglement_sizes", _sz, [_vp, ctypes.POINTER(_sz)]),
    ("ecut_entanglement_spectrum", _i32, [_vp, _vp, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.POINTER(Entanglement), _vp, _vp]),
    ("ecut_server_create", _i32, [_sz, ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]),
    ("ecut_server_submit", _i32, [_vp, ctypes.POINTER(ModelDesc), ctypes.POINTER(CutDesc), QNum, _u64, _dbl,
                                  ctypes.POINTER(_u64)]),
    ("ecut_server_poll", _i32, [_vp, ctypes.POINTER(Result), _i32, ctypes.POINTER(_i32)]),
    ("ecut_server_drain", _i32, [_vp]),
    ("ecut_server_now", _dbl, [_vp]),
    ("ecut_server_destroy", None, [_vp]),
    ("ecut_set_allocator", _i32, [ALLOC_FN, FREE_FN, _vp]),
    ("ecut_last_error", ctypes.c_char_p, []),
    ("ecut_version", ctypes.c_char_p, []),
]

_lib = None
_allocators = []   # every pair ever installed: blocks they made are released through them


def lib():
    """Load libecut.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              f"(or python paper_2605_07621_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SYMBOLS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != ECUT_OK:
        raise EcutError(st, lib().ecut_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return _vp(stream.cuda_stream)
    return _vp(stream)


def _dptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    return _vp(t.data_ptr())


class _ModelArgs:
    """Keeps the numpy arrays alive behind a ModelDesc / CutDesc / QNum."""

    def __init__(self, model, cut, n_up, n_dn=0):
        b = np.ascontiguousarray(np.asarray(model.bonds, dtype=np.int32).reshape(-1, 2))
        self.bi = np.ascontiguousarray(b[:, 0])
        self.bj = np.ascontiguousarray(b[:, 1])
        nb = len(self.bi)
        p = lambda a: None if a is None else a.ctypes.data
        if model.kind == "spin":
            self.jxy = np.ascontiguousarray(model.jxy, dtype=np.float64)
            self.jz = np.ascontiguousarray(model.jz, dtype=np.float64)
            self.t = self.u = self.v = None
            kind = ECUT_SPIN_HALF
        elif model.kind == "hubbard":
            self.t = np.ascontiguousarray(model.t, dtype=np.float64)
            self.u = None if model.u is None else np.ascontiguousarray(model.u, dtype=np.float64)
            v = getattr(model, "v", None)
            self.v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
            self.jxy = self.jz = None
            kind = ECUT_HUBBARD
        else:
            raise ValueError(f"unknown model kind {model.kind!r}")
        self.m = ModelDesc(kind, int(model.n_sites), nb, 0, p(self.bi), p(self.bj), p(self.jxy), p(self.jz),
                           p(self.t), p(self.u), p(self.v))
        ck = {"spatial": ECUT_CUT_SPATIAL, "updn": ECUT_CUT_UPDN}.get(cut.kind)
        if ck is None:
            raise ValueError(f"unknown cut kind {cut.kind!r}")
        self.c = CutDesc(ck, 0, int(cut.left_mask))
        self.q = QNum(int(n_up), int(n_dn))


class Sectors:
    """ecut_sectors handle: the bipartite description of H in one sector."""

    def __init__(self, model, cut, n_up, n_dn=0, host_only=False):
        self._args = _ModelArgs(model, cut, n_up, n_dn)
        h = _vp()
        _check(lib().ecut_build_sectors(ctypes.byref(self._args.m), ctypes.byref(self._args.c), self._args.q,
                                        ECUT_BUILD_HOST_ONLY if host_only else 0, ctypes.byref(h)))
        self.h = h
        i = SectorsInfo()
        _check(lib().ecut_sectors_get_info(self.h, ctypes.byref(i)))
        self.info = i
        self.dim = int(i.dim)

    @classmethod
    def from_problem(cls, p, host_only=False):
        return cls(p.model, p.cut, p.n_up, p.n_dn, host_only=host_only)

    def close(self):
        if getattr(self, "h", None):
            lib().ecut_sectors_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def blocks(self):
        out = np.empty(5 * self.info.n_blocks, dtype=np.int64)
        _check(lib().ecut_sectors_blocks(self.h, out.ctypes.data))
        return out.reshape(-1, 5)

    def words(self, block):
        b = self.blocks()[block]
        lw = np.empty(int(b[2]), dtype=np.uint32)
        rw = np.empty(int(b[3]), dtype=np.uint32)
        _check(lib().ecut_sectors_words(self.h, int(block), lw.ctypes.data, rw.ctypes.data))
        return lw, rw

    def canonical_positions(self):
        pos = np.empty(self.dim, dtype=np.int64)
        _check(lib().ecut_canonical_positions(self.h, pos.ctypes.data))
        return pos

    def canonical_signs(self):
        sg = np.empty(self.dim, dtype=np.int8)
        _check(lib().ecut_canonical_signs(self.h, _vp(sg.ctypes.data)))
        return sg

    def labels(self):
        lab = np.empty((self.info.n_blocks, 4), dtype=np.int32)
        _check(lib().ecut_sectors_labels(self.h, _vp(lab.ctypes.data)))
        return lab

    def import_(self, canon, out=None, stream=None):
        import torch
        out = torch.empty(self.dim, dtype=torch.float64, device=canon.device) if out is None else out
        _check(lib().ecut_import(self.h, _dptr(canon, self.dim, "canon"), _dptr(out, self.dim, "out"), _stream(stream)))
        return out

    def export(self, bip, out=None, stream=None):
        import torch
        out = torch.empty(self.dim, dtype=torch.float64, device=bip.device) if out is None else out
        _check(lib().ecut_export(self.h, _dptr(bip, self.dim, "bip"), _dptr(out, self.dim, "out"), _stream(stream)))
        return out

    def apply(self, psi, out=None, stream=None):
        import torch
        out = torch.empty(self.dim, dtype=torch.float64, device=psi.device) if out is None else out
        _check(lib().ecut_apply_H(self.h, _dptr(psi, self.dim, "psi"), _dptr(out, self.dim, "out"), _stream(stream)))
        return out

    def entanglement(self, psi, n_parts=1, part_of_block=None, cutoff=1e-14, stream=None):
        """ecut_entanglement_spectrum: dict of lambda, xi (per block, lists of
        numpy arrays), w_q, chi_q, w_p and the summary fields."""
        import numpy as np
        import torch
        nl = _sz()
        nws = int(lib().ecut_entanglement_sizes(self.h, ctypes.byref(nl)))
        ws = torch.empty(nws, dtype=torch.float64, device=psi.device)
        nb = self.info.n_blocks
        lam = np.empty(nl.value)
        xi = np.empty(nl.value)
        wq = np.empty(nb)
        chi = np.empty(nb, dtype=np.int32)
        wp = np.empty(int(n_parts))
        pob = None if part_of_block is None else np.ascontiguousarray(part_of_block, dtype=np.int32)
        summ = Entanglement()
        _check(lib().ecut_entanglement_spectrum(self.h, _dptr(psi, self.dim, "psi"), float(cutoff), int(n_parts),
                                                None if pob is None else _vp(pob.ctypes.data),
                                                _vp(lam.ctypes.data), _vp(xi.ctypes.data), _vp(wq.ctypes.data),
                                                _vp(chi.ctypes.data), _vp(wp.ctypes.data), ctypes.byref(summ),
                                                _dptr(ws, nws, "workspace"), _stream(stream)))
        b = self.blocks()
        m = np.minimum(b[:, 2], b[:, 3])
        cut = np.concatenate([[0], np.cumsum(m)])
        return dict(lam=[lam[cut[q]:cut[q + 1]] for q in range(nb)], xi=[xi[cut[q]:cut[q + 1]] for q in range(nb)],
                    w_q=wq, chi_q=chi, w_p=wp, norm2=summ.norm2, weight_ipr=summ.weight_ipr, n_eff=summ.n_eff,
                    entropy=summ.entropy)

    def get_tuning(self):
        t = Tuning()
        _check(lib().ecut_get_tuning(self.h, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, grid=0, n_xcd=0, row_order=0, variant=0, tile=0):
        t = Tuning(int(grid), int(n_xcd), int(row_order), int(variant), int(tile))
        _check(lib().ecut_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, x, y, stream=None):
        t = Tuning()
        _check(lib().ecut_autotune(self.h, _dptr(x, self.dim, "x"), _dptr(y, self.dim, "y"), _stream(stream),
                                   ctypes.byref(t)))
        return _tuning_dict(t)

    def lanczos_workspace(self, max_steps, reorth=False, max_restarts=0, tol=1e-10, fixed_steps=False):
        o = LanczosOpts(int(max_steps), int(max_restarts), int(bool(reorth)), int(bool(fixed_steps)), float(tol))
        return int(lib().ecut_lanczos_workspace(self.h, ctypes.byref(o)))

    def lanczos(self, v0, max_steps, tol=1e-10, reorth=False, fixed_steps=False, max_restarts=0,
                want_gs=False, workspace=None, stream=None, allow_notconv=False, use_graph=False):
        """Returns (energy, stats dict, ground state or None)."""
        import torch
        o = LanczosOpts(int(max_steps), int(max_restarts), int(bool(reorth)), int(bool(fixed_steps)), float(tol),
                        int(bool(use_graph)))
        nws = int(lib().ecut_lanczos_workspace(self.h, ctypes.byref(o)))
        ws = torch.empty(nws, dtype=torch.float64, device=v0.device) if workspace is None else workspace
        gs = torch.empty(self.dim, dtype=torch.float64, device=v0.device) if want_gs else None
        e = _dbl()
        stt = LanczosStats()
        st = lib().ecut_lanczos_ground_state(self.h, _dptr(v0, self.dim, "v0"), ctypes.byref(o), ctypes.byref(e),
                                             None if gs is None else _vp(gs.data_ptr()), ctypes.byref(stt),
                                             _dptr(ws, nws, "workspace"), _stream(stream))
        if not (st == ECUT_OK or (allow_notconv and st == ECUT_ENOTCONV)):
            _check(st)
        stats = dict(steps=stt.steps, restarts=stt.restarts, converged=stt.converged, residual=stt.residual,
                     seconds=stt.seconds, status=st)
        return e.value, stats, gs


def apply_cdag(src, dst, site, spin, dagger, x, out=None, stream=None):
    """ecut_apply_cdag: c+ (dagger) or c of mode (site, spin) from sector
    src to sector dst (bipartite layouts of each)."""
    import torch
    y = torch.empty(dst.dim, dtype=torch.float64, device=x.device) if out is None else out
    _check(lib().ecut_apply_cdag(src.h, dst.h, int(site), int(spin), 1 if dagger else 0, _dptr(x, src.dim, "x"),
                                 _dptr(y, dst.dim, "y"), _stream(stream)))
    return y


def lanczos_tridiag(S, v0, n_steps, stream=None):
    """ecut_lanczos_tridiag: (alpha, beta, |v0|^2) of n_steps Lanczos steps
    of S's H from v0."""
    import numpy as np
    import torch
    o = LanczosOpts(int(n_steps), 0, 0, 1, 1e-10, 0)
    nws = int(lib().ecut_lanczos_workspace(S.h, ctypes.byref(o)))
    ws = torch.empty(nws, dtype=torch.float64, device=v0.device)
    a = np.zeros(n_steps)
    b = np.zeros(n_steps)
    n = _i32()
    nrm = _dbl()
    _check(lib().ecut_lanczos_tridiag(S.h, _dptr(v0, S.dim, "v0"), int(n_steps), _vp(a.ctypes.data), _vp(b.ctypes.data),
                                      ctypes.byref(n), ctypes.byref(nrm), _dptr(ws, nws, "workspace"), _stream(stream)))
    return a[:n.value].copy(), b[:n.value].copy(), nrm.value


def continued_fraction(alpha, beta, weight, e0, dagger, omega, eta):
    """ecut_continued_fraction: complex numpy array of G(omega)."""
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(omega, dtype=np.float64)
    re = np.empty(len(w))
    im = np.empty(len(w))
    _check(lib().ecut_continued_fraction(_vp(a.ctypes.data), _vp(b.ctypes.data), len(a), float(weight), float(e0),
                                         1 if dagger else 0, _vp(w.ctypes.data), len(w), float(eta),
                                         _vp(re.ctypes.data), _vp(im.ctypes.data)))
    return re + 1j * im


def green_function(S0, gs, e0, S1, site, spin, dagger, n_steps, omega, eta, stream=None):
    """G+(omega) (dagger) or G-(omega) of mode (site, spin) on the ground
    state gs (bipartite layout of S0, energy e0), with S1 the sector of
    c+ gs (resp. c gs): apply_cdag, lanczos_tridiag and continued_fraction
    of the library in turn.  Returns (G, alpha, beta, weight)."""
    y = apply_cdag(S0, S1, site, spin, dagger, gs, stream=stream)
    a, b, w = lanczos_tridiag(S1, y, n_steps, stream=stream)
    return continued_fraction(a, b, w, e0, dagger, omega, eta), a, b, w


def set_allocator(alloc=None, free=None):
    """ecut_set_allocator: alloc(nbytes, device) -> device address (int, 0 on
    failure) and free(ptr, nbytes, device) back the sector tables of handles
    built from now on; set_allocator() restores hipMalloc / hipFree.  The
    callbacks are kept alive for the life of the process."""
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both be None")
    if alloc is None:
        _check(lib().ecut_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    a = ALLOC_FN(lambda nbytes, device, user: alloc(nbytes, device) or None)
    f = FREE_FN(lambda ptr, nbytes, device, user: free(ptr, nbytes, device))
    _allocators.append((a, f))
    _check(lib().ecut_set_allocator(a, f, None))


def torch_allocator():
    """An (alloc, free) pair for set_allocator backed by torch's CUDA caching
    allocator (on the current stream of the device at allocation)."""
    import torch

    def alloc(nbytes, device):
        return torch.cuda.caching_allocator_alloc(nbytes, device)

    def free(ptr, nbytes, device):
        torch.cuda.caching_allocator_delete(ptr)

    return alloc, free


def apply_batch(sectors, psis, ys, stream=None, noalloc=False):
    """ecut_apply_H_batch, or ecut_apply_H_batch_noalloc with noalloc=True."""
    n = len(sectors)
    hs = (_vp * n)(*[s.h for s in sectors])
    ps = (_vp * n)(*[_dptr(p, s.dim, "psi") for s, p in zip(sectors, psis)])
    qs = (_vp * n)(*[_dptr(y, s.dim, "y") for s, y in zip(sectors, ys)])
    f = lib().ecut_apply_H_batch_noalloc if noalloc else lib().ecut_apply_H_batch
    _check(f(n, ctypes.cast(hs, _vp), ctypes.cast(ps, _vp), ctypes.cast(qs, _vp), _stream(stream)))


class Server:
    """Continuous-batching ground-state server (ecut_server_*)."""

    def __init__(self, hbm_budget, max_active=0, max_steps=400, tol=1e-10, sequential=False, use_graph=False,
                 autotune=False, large_dim=0):
        o = ServerOpts(int(max_active), int(max_steps), float(tol), int(bool(sequential)), int(bool(use_graph)),
                       int(bool(autotune)), int(large_dim))
        h = _vp()
        _check(lib().ecut_server_create(int(hbm_budget), ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, problem, seed, not_before=0.0):
        a = _ModelArgs(problem.model, problem.cut, problem.n_up, problem.n_dn)
        rid = _u64()
        _check(lib().ecut_server_submit(self.h, ctypes.byref(a.m), ctypes.byref(a.c), a.q, int(seed),
                                        float(not_before), ctypes.byref(rid)))
        return int(rid.value)

    def poll(self, max_results=1024):
        buf = (Result * max_results)()
        n = _i32()
        st = lib().ecut_server_poll(self.h, buf, max_results, ctypes.byref(n))
        if st not in (ECUT_OK, ECUT_EAGAIN):
            _check(st)
        return [dict(req_id=r.req_id, status=r.status, steps=r.steps, energy=r.energy, residual=r.residual,
                     t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done) for r in buf[:n.value]]

    def drain(self):
        _check(lib().ecut_server_drain(self.h))

    def now(self):
        return lib().ecut_server_now(self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().ecut_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
