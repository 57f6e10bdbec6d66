"""GPU parity of the bipartite H*psi, the Lanczos solver, batching and
serving against the CPU oracle.  All calls go through the C ABI (ctypes
binding); the oracle sees the same seeded canonical-order inputs.

Tolerance: H*psi relative L2 error <= 1e-12 (and every element within
1e-12 * max|y|); ground energies within 1e-10 absolute."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2605_07621_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def _ecut():
    from paper_2605_07621_amd import ecut
    return ecut


def _compare(y, y_ref, what):
    err = np.linalg.norm(y - y_ref) / max(np.linalg.norm(y_ref), 1e-300)
    assert err <= RTOL, f"{what}: relative L2 {err:.3e}"
    assert np.max(np.abs(y - y_ref)) <= RTOL * max(np.max(np.abs(y_ref)), 1e-300) * 10, what


def _gpu_apply_canonical(S, psi, dev):
    import torch
    x = S.import_(torch.from_numpy(psi).to(dev))
    y = S.apply(x)
    out = S.export(y).cpu().numpy()
    torch.cuda.synchronize()
    return out


SMALL = []
_rng = np.random.default_rng(2024)
for n, mask in [(8, 0b00001111), (10, 0b1001010110), (11, 0b1), (9, 0b111111110), (12, 0b101010101010)]:
    m = I.random_spin_model(_rng, n, n_bonds=2 * n)
    for n_up in sorted({0, 1, n // 2, n - 1}):
        SMALL.append(I.Problem(m, I.Cut("spatial", mask), n_up))
SMALL.append(I.Problem(I.xxz_chain(7, 1.0, 1.0), I.Cut("spatial", 0), 3))
SMALL.append(I.Problem(I.xxz_chain(7, 1.0, 1.0), I.Cut("spatial", 0x7f), 3))
for L in (4, 6, 8, 10):
    hm = I.random_hubbard_model(_rng, L, n_bonds=2 * L)
    SMALL.append(I.Problem(hm, I.Cut("updn"), L // 2, L // 2 - 1))
    SMALL.append(I.Problem(I.hubbard_chain(L, 1.0, 3.5), I.Cut("updn"), L // 2, L // 2))
SMALL.append(I.Problem(I.hubbard_chain(5, 1.0, 2.0), I.Cut("updn"), 0, 2))
SMALL.append(I.Problem(I.hubbard_chain(5, 1.0, 2.0), I.Cut("updn"), 5, 5))


@pytest.mark.parametrize("k", range(len(SMALL)))
def test_apply_small_vs_oracle(dev, k):
    p = SMALL[k]
    s = O.Sector(p.model, p.n_up, p.n_dn)
    psi = I.psi(100 + k, s.n)
    y_ref = s.apply(psi)
    S = _ecut().Sectors.from_problem(p)
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{p.model.name} n_up={p.n_up}")


_WIDE = [
    # Hubbard beyond the up/down kernels' 20-site tables: the generic row kernel
    I.Problem(I.hubbard_chain(22, 1.0, 3.0, periodic=True), I.Cut("updn"), 2, 1),
    I.Problem(I.random_hubbard_model(np.random.default_rng(31), 24, n_bonds=40), I.Cut("updn"), 1, 2),
    # Hubbard with class tiles but no whole-row kernel (more than 16 sites)
    I.Problem(I.hubbard_chain(18, 0.8, 5.0), I.Cut("updn"), 2, 3),
    # spin models with a side wider than 16 sites (generic row kernel)
    I.Problem(I.xxz_chain(40, 1.0, 0.7, periodic=True), I.Cut("spatial", (1 << 20) - 1), 2),
    I.Problem(I.random_spin_model(np.random.default_rng(32), 34, n_bonds=50), I.Cut("spatial", (1 << 17) - 1), 3),
]


@pytest.mark.parametrize("k", range(len(_WIDE)))
def test_apply_wide_lattices_vs_oracle(dev, k):
    """Lattices wider than the specialised kernels take (and must agree on)
    the generic paths; the whole-row Hubbard kernel is refused there."""
    p = _WIDE[k]
    s = O.Sector(p.model, p.n_up, p.n_dn)
    psi = I.psi(800 + k, s.n)
    y_ref = s.apply(psi)
    S = _ecut().Sectors.from_problem(p)
    assert not S.info.kernel_flags & (4 | 8)
    if p.model.kind == "hubbard" and S.info.kernel == 1:
        with pytest.raises(_ecut().EcutError):
            S.set_tuning(0, 1, 0, 4)
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{p.model.name} n_up={p.n_up} n_dn={p.n_dn}")


_HUB_CASES = [I.hubbard12(),
              I.Problem(I.hubbard_chain(10, 1.0, 2.5), I.Cut("updn"), 5, 4),
              I.Problem(I.hubbard_chain(11, 0.7, 6.0), I.Cut("updn"), 6, 3),
              I.Problem(I.random_hubbard_model(np.random.default_rng(77), 9, n_bonds=14), I.Cut("updn"), 4, 5),
              I.Problem(I.random_hubbard_model(np.random.default_rng(78), 10, n_bonds=12), I.Cut("updn"), 3, 5)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("order", [0, 2, 4, 7, 9])
def test_hubbard_kernel_variants_and_orders(dev, variant, order):
    """Every Hubbard kernel (class tiles with the uniform-chain fast path,
    whole rows in LDS, generic class tiles, two passes, whole rows with
    16-byte access and ranked hops, segment tiles, two passes on flat items)
    under several work orders agrees with the oracle; uniform chains and
    random long-range couplings (fermion signs), even and odd row lengths."""
    for k, p in enumerate(_HUB_CASES):
        s = O.Sector(p.model, p.n_up, p.n_dn)
        psi = I.psi(500 + k, s.n)
        y_ref = s.apply(psi)
        S = _ecut().Sectors.from_problem(p)
        if variant == 4 and not S.info.kernel_flags & 8:
            assert math.comb(p.model.n_sites, p.n_dn) % 2 == 1
            with pytest.raises(_ecut().EcutError):
                S.set_tuning(0, 1, order, variant)
            continue
        if variant == 3 and not S.info.kernel_flags & 2:
            with pytest.raises(_ecut().EcutError):
                S.set_tuning(0, 1, order, variant)
            continue
        if variant == 6:
            assert S.info.kernel_flags & 32   # every up/down problem takes the two-pass kernels
        if variant == 7 and not S.info.kernel_flags & 2:
            with pytest.raises(_ecut().EcutError):
                S.set_tuning(0, 1, order, variant)
            continue
        if variant == 5 and not S.info.kernel_flags & 16:
            assert not S.info.kernel_flags & 2    # segment tiles cover every uniform sign-free chain here
            with pytest.raises(_ecut().EcutError):
                S.set_tuning(0, 1, order, variant)
            continue
        S.set_tuning(0, 8 if order % 2 == 0 else 1, order, variant)
        assert S.get_tuning()["variant"] == variant
        _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{p.model.name} v{variant} o{order}")


def test_hubbard_two_pass_item_shapes_bit_exact(dev):
    """The two-pass kernels (variant 6) give the same vector bit for bit for
    every rows-per-item tile of either pass, XCD chunking and row order (each
    amplitude is summed in the same order whatever the item shape), the
    oracle's vector;
    in Lanczos steps the per-item partials follow the item split and the
    energy stays the oracle's.  Cases: uniform chains (no hop values stored),
    random long-range hoppings with fermion signs and site-dependent U, odd
    row lengths (one column per lane), a 1 x n and an n x 1 block."""
    import torch
    E = _ecut()
    cases = list(_HUB_CASES) + [I.Problem(I.hubbard_chain(7, 1.0, 2.0), I.Cut("updn"), 0, 3),
                                I.Problem(I.hubbard_chain(7, 1.0, 2.0), I.Cut("updn"), 4, 7)]
    for k, p in enumerate(cases):
        s = O.Sector(p.model, p.n_up, p.n_dn)
        psi = I.psi(1500 + k, s.n)
        y_ref = s.apply(psi)
        S = E.Sectors.from_problem(p)
        assert S.info.kernel_flags & 32
        x = S.import_(torch.from_numpy(psi).to(dev))
        y0 = None
        for tile, left in ((1, 0), (2, 4), (4, 0), (8, 16), (16, 1)):
            for xcd, order in ((8, 0), (1, 1), (8, 2)):
                # left: rows per item of the left-operator pass (0 = default)
                S.set_tuning(left, xcd, order, 6, tile)
                y = S.apply(x)
                torch.cuda.synchronize()
                if y0 is None:
                    y0 = y
                    _compare(S.export(y).cpu().numpy(), y_ref, f"{p.model.name} two-pass")
                assert torch.equal(y, y0), (p.model.name, tile, xcd, order)
        if s.n >= 64:
            e_ref = s.lanczos(I.psi(1600 + k, s.n), 400, tol=1e-14)[0][-1]
            v0 = S.import_(torch.from_numpy(I.psi(1600 + k, s.n)).to(dev))
            for tile in (1, 16):
                S.set_tuning(0, 8, 1, 6, tile)
                ws = torch.full((S.lanczos_workspace(400, tol=1e-11),), float("nan"), dtype=torch.float64, device=dev)
                e, st, _ = S.lanczos(v0, 400, tol=1e-11, workspace=ws)
                assert st["converged"] and abs(e - e_ref) <= 1e-10, (p.model.name, tile, e, e_ref)


def test_hubbard_whole_row_group_sizes(dev):
    """The whole-row kernel (variant 4) with 256-, 512- and 1024-thread work
    groups gives the same vector bit for bit, the oracle's on the small cases;
    the 14-site chain (rows of 3,432 columns) runs at every group size."""
    import torch
    E = _ecut()
    cases = list(_HUB_CASES) + [I.Problem(I.hubbard_chain(14, 1.0, 4.0), I.Cut("updn"), 7, 7)]
    for k, p in enumerate(cases):
        S = E.Sectors.from_problem(p)
        if not S.info.kernel_flags & 8:
            continue
        d_r = int(S.blocks()[0][3])
        x = torch.from_numpy(I.psi(600 + k, S.dim)).to(dev)
        ys = {}
        for threads in (1024, 512, 256):
            if d_r > 14 * threads:
                with pytest.raises(E.EcutError):
                    S.set_tuning(0, 8, 0, 4, threads)
                continue
            S.set_tuning(0, 8, 9 if threads == 256 else 0, 4, 0 if threads == 1024 else threads)
            ys[threads] = S.apply(x).cpu()
        assert 256 in ys or d_r > 14 * 256
        for threads, y in ys.items():
            assert torch.equal(y, ys[1024]), (p.model.name, threads)
        if S.dim <= 1 << 20:
            s = O.Sector(p.model, p.n_up, p.n_dn)
            psi = I.psi(700 + k, s.n)
            S.set_tuning(0, 1, 0, 4, 256 if d_r <= 14 * 256 else 0)
            _compare(_gpu_apply_canonical(S, psi, dev), s.apply(psi), f"{p.model.name} whole rows, small groups")


@pytest.mark.parametrize("name", ["heisenberg16", "hubbard12"])
def test_apply_workload_full_vs_oracle(dev, name):
    p = I.WORKLOADS[name]()
    s = O.Sector(p.model, p.n_up, p.n_dn)
    psi = I.psi(p.meta["seed"], s.n)
    y_ref = s.apply(psi)
    S = _ecut().Sectors.from_problem(p)
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, name)


def _full_size_setup(name, dev):
    """Sector handle autotuned on the workload's input (the launch
    configuration the benchmark times), the oracle's sector and the input."""
    import torch
    p = I.WORKLOADS[name]()
    sec = O.Sector(p.model, p.n_up, p.n_dn)
    psi = I.psi(p.meta["seed"], sec.n)
    S = _ecut().Sectors.from_problem(p)
    xt = S.import_(torch.from_numpy(psi).to(dev))
    tuned = S.autotune(xt, torch.empty_like(xt))
    del xt
    return p, sec, psi, S, tuned


def _compare_full(y, y_ref, what):
    """Whole-vector element-wise comparison (relative L2 and max error)."""
    d = y - y_ref
    err = np.linalg.norm(d) / np.linalg.norm(y_ref)
    big = np.max(np.abs(d)) / np.max(np.abs(y_ref))
    print(f"[full] {what}: relative L2 {err:.2e}, max {big:.2e}", flush=True)
    assert err <= RTOL, f"{what}: relative L2 {err:.3e}"
    assert big <= RTOL * 10, f"{what}: max element error {big:.3e}"


# Hubbard kernels at full size, each compared with the oracle's whole vector:
# (grid, n_xcd, row order, variant, tile)
_FULL_HUB_TUNINGS = ((0, 8, 8, 0, 0), (0, 8, 7, 0, 0), (0, 1, 1, 4, 0), (0, 8, 2, 4, 0), (0, 8, 0, 5, 0),
                     (0, 8, 8, 7, 0), (8, 8, 7, 7, 0), (0, 8, 1, 6, 4), (4, 1, 0, 6, 2), (16, 8, 2, 6, 8))


def test_apply_full_size_hubbard16_whole_vector_vs_oracle(dev):
    """16-site Hubbard chain, 165,636,900 amplitudes: the whole H*psi vector
    of the autotuned launch configuration, and of every Hubbard kernel
    variant, compared element by element with the oracle's (rows of the full
    occupation-basis H, no stored matrix), plus Hermiticity on the device."""
    import time
    import torch
    p, sec, psi, S, tuned = _full_size_setup("hubbard16", dev)
    print(f"[full] hubbard16 autotuned {tuned}", flush=True)
    t0 = time.time()
    y_ref = sec.apply(psi, use_csr=False)
    print(f"[full] oracle apply {time.time() - t0:.1f} s on {O.num_threads()} threads", flush=True)
    _compare_full(_gpu_apply_canonical(S, psi, dev), y_ref, f"autotuned {tuned}")
    for t in _FULL_HUB_TUNINGS:
        S.set_tuning(*t)
        _compare_full(_gpu_apply_canonical(S, psi, dev), y_ref, f"tuning {t}")
    x = torch.from_numpy(psi).to(dev)
    phi = torch.from_numpy(I.psi(p.meta["seed"] + 2, sec.n)).to(dev)
    xb, pb = S.import_(x), S.import_(phi)
    lhs = torch.dot(pb, S.apply(xb)).item()
    rhs = torch.dot(S.apply(pb), xb).item()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_apply_full_size_j1j2_blocks_vs_oracle(dev):
    """6x5 J1-J2 lattice, 155,117,520 amplitudes in 16 blocks: in the
    autotuned launch configuration, every amplitude of the largest block
    (6,435 x 6,435 = 41.4M) and of blocks 0, 1, 14 and 15 against the
    oracle's rows, the blocks found through the
    oracle's own bipartite map; Hermiticity on the device."""
    import time
    import torch
    p, sec, psi, S, tuned = _full_size_setup("j1j2_6x5", dev)
    print(f"[full] j1j2_6x5 autotuned {tuned}", flush=True)
    y = _gpu_apply_canonical(S, psi, dev)
    pos, blocks = sec.bipartite(p.cut.kind, p.cut.left_mask)
    sizes = blocks[:, 1] * blocks[:, 2]
    big = int(np.argmax(sizes))
    for b in sorted({0, 1, big, len(blocks) - 2, len(blocks) - 1}):
        off, n_b = int(blocks[b, 3]), int(sizes[b])
        rows = np.nonzero((pos >= off) & (pos < off + n_b))[0]
        assert len(rows) == n_b
        t0 = time.time()
        y_ref = sec.apply_rows(psi, rows)
        print(f"[full] block {b}: {n_b} rows, oracle {time.time() - t0:.1f} s", flush=True)
        _compare_full(y[rows], y_ref, f"j1j2 block {b}")
        del rows, y_ref
    del pos
    x = torch.from_numpy(psi).to(dev)
    phi = torch.from_numpy(I.psi(p.meta["seed"] + 2, sec.n)).to(dev)
    xb, pb = S.import_(x), S.import_(phi)
    lhs = torch.dot(pb, S.apply(xb)).item()
    rhs = torch.dot(S.apply(pb), xb).item()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_cut_invariance_heisenberg16(dev):
    """H*psi brought back to canonical order does not depend on where the
    chain is cut: every cut 1|15 ... 15|1 gives the oracle's vector."""
    p = I.heisenberg16()
    s = O.Sector(p.model, p.n_up)
    psi = I.psi(p.meta["seed"], s.n)
    y_ref = s.apply(psi)
    for k in range(1, 16):
        S = _ecut().Sectors.from_problem(I.Problem(p.model, I.Cut("spatial", (1 << k) - 1), p.n_up))
        _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"cut {k}|{16 - k}")


def test_cut_invariance_j1j2_6x5_full_size(dev):
    """At full size (155M amplitudes) the 6x5 J1-J2 apply gives the same
    canonical vector for the x<=2 | x>=3 cut, its mirror, and a checkerboard
    cut whose 49 nearest-neighbour bonds all cross it."""
    import torch
    p = I.j1j2_6x5()
    full = (1 << 30) - 1
    checker = sum(1 << (5 * x + y) for x in range(6) for y in range(5) if (x + y) % 2 == 0)
    x = torch.from_numpy(I.psi(p.meta["seed"] + 9, math.comb(30, 15))).to(dev)
    ref = None
    for mask in (p.cut.left_mask, full ^ p.cut.left_mask, checker):
        S = _ecut().Sectors.from_problem(I.Problem(p.model, I.Cut("spatial", mask), p.n_up))
        assert S.info.kernel_flags & 4
        xt = S.import_(x)
        S.autotune(xt, torch.empty_like(xt))
        y = S.export(S.apply(xt))
        del xt
        torch.cuda.synchronize()
        if ref is None:
            ref = y
            continue
        err = (torch.linalg.vector_norm(y - ref) / torch.linalg.vector_norm(ref)).item()
        assert err <= RTOL, (hex(mask), err)
        del y


def test_hubbard16_spin_flip_symmetry_full_size(dev):
    """With N_up = N_dn the Hamiltonian is symmetric under exchanging the
    spins, so H (Psi^T) = (H Psi)^T for the 12,870 x 12,870 canonical
    amplitude matrix, in the autotuned launch configuration."""
    import torch
    p = I.hubbard16()
    S = _ecut().Sectors.from_problem(p)
    n = math.comb(16, 8)
    x = torch.from_numpy(I.psi(p.meta["seed"] + 7, S.dim)).to(dev)
    xi = S.import_(x)
    S.autotune(xi, torch.empty_like(xi))
    y = S.export(S.apply(xi)).view(n, n)
    del xi
    xt = x.view(n, n).t().contiguous().view(-1)
    del x
    yt = S.export(S.apply(S.import_(xt))).view(n, n)
    torch.cuda.synchronize()
    err = (torch.linalg.vector_norm(yt - y.t()) / torch.linalg.vector_norm(y)).item()
    assert err <= RTOL, err


def test_apply_is_deterministic_and_batch_bit_exact(dev):
    import torch
    ecut = _ecut()
    probs = [SMALL[3], SMALL[9], I.heisenberg16(), I.hubbard12(), SMALL[-3]]
    Ss = [ecut.Sectors.from_problem(p) for p in probs]
    xs = [torch.from_numpy(I.psi(300 + k, S.dim)).to(dev) for k, S in enumerate(Ss)]
    alone = [S.apply(x) for S, x in zip(Ss, xs)]
    again = [S.apply(x) for S, x in zip(Ss, xs)]
    ys = [torch.empty_like(x) for x in xs]
    ecut.apply_batch(Ss, xs, ys)
    torch.cuda.synchronize()
    for k in range(len(Ss)):
        assert torch.equal(alone[k], again[k])
        assert torch.equal(alone[k], ys[k]), f"batch differs for problem {k}"


_SPIN_CASES = [p for p in SMALL if p.model.kind == "spin"] + [
    I.heisenberg16(),
    I.Problem(I.xxz_chain(20, 1.0, 0.6), I.Cut("spatial", (1 << 10) - 1), 10),
    I.Problem(I.j1j2_lattice(4, 3, 1.0, 0.5), I.Cut("spatial", (1 << 6) - 1), 6),
    I.Problem(I.j1j2_lattice(4, 4, 1.0, 0.5), I.Cut("spatial", 0b1010101101010110), 7),
    I.Problem(I.random_spin_model(np.random.default_rng(91), 16, n_bonds=60), I.Cut("spatial", 0x0f0f), 8),
    # the diagonal cross terms' right sites are not one bit field of the right
    # word (positions 0, 4, 5): the kernels gather the bits into the table index
    I.Problem(I.xxz_chain(20, 1.0, 1.3), I.Cut("spatial", 0x7C1F), 10),
    # nine distinct right sites, more than the folded table takes: the terms
    # are summed one by one
    I.Problem(I.random_spin_model(np.random.default_rng(93), 18, n_bonds=90), I.Cut("spatial", (1 << 9) - 1), 9),
]


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_spin_kernel_variants(dev, variant):
    """The ranking-table spin kernel (variant 0), the generic row kernel
    (variant 1) and the two-pass spin kernels (variant 2) all agree with the
    oracle: Heisenberg, XXZ and J1-J2 models, random couplings and cuts,
    one-row and many-row tiles, empty and full sectors."""
    for k, p in enumerate(_SPIN_CASES):
        s = O.Sector(p.model, p.n_up, p.n_dn)
        psi = I.psi(700 + k, s.n)
        y_ref = s.apply(psi)
        S = _ecut().Sectors.from_problem(p)
        if variant == 2 and not S.info.kernel_flags & 64:
            continue
        S.set_tuning(0, 0, 0, variant)
        assert S.get_tuning()["variant"] == variant
        _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{p.model.name} n_up={p.n_up} variant {variant}")


def test_spin_kernel_full_size_variants_agree(dev):
    """At the 6x5 J1-J2 size (16 blocks, 155M amplitudes) the spin kernel
    and the generic row kernel give the same vector to 1e-12."""
    import torch
    p = I.j1j2_6x5()
    S = _ecut().Sectors.from_problem(p)
    assert S.info.kernel_flags & 4
    x = torch.from_numpy(I.psi(p.meta["seed"] + 3, S.dim)).to(dev)
    S.set_tuning(0, 0, 0, 0)
    y0 = S.apply(x)
    S.set_tuning(0, 0, 0, 1)
    y1 = S.apply(x)
    torch.cuda.synchronize()
    err = (torch.linalg.vector_norm(y0 - y1) / torch.linalg.vector_norm(y1)).item()
    assert err <= RTOL, err
    # the autotuner times each candidate with its own kernel: a spin kernel
    # is several times faster here than the generic one, so it must win
    assert S.autotune(x, y1)["variant"] in (0, 2)
    del y0, y1, x


def test_spin_two_pass_bit_exact(dev):
    """The two-pass spin kernels sum every amplitude's terms in the spin
    kernel's order (left operator in CSR order, then cross terms, right
    operator, diagonal), so every left-pass row count, XCD dealing and
    short-row tile gives the one-pass vector bit for bit; and the oracle's."""
    import torch
    n_run = 0
    for k, p in enumerate(_SPIN_CASES):
        S = _ecut().Sectors.from_problem(p)
        if not S.info.kernel_flags & 64:
            continue
        s = O.Sector(p.model, p.n_up, p.n_dn)
        psi = I.psi(1500 + k, s.n)
        x = S.import_(torch.from_numpy(psi).to(dev))
        S.set_tuning(0, 0, 0, 0, 0)
        y0 = S.apply(x)
        for rows, xcd, tile in ((0, 8, 0), (4, 1, 0), (8, 8, 64), (16, 8, 1), (32, 1, 512), (5, 8, 300)):
            S.set_tuning(rows, xcd, 0, 2, tile)
            y = S.apply(x)
            torch.cuda.synchronize()
            assert torch.equal(y, y0), f"{p.model.name} n_up={p.n_up} rows {rows} xcd {xcd} tile {tile}"
        _compare(_gpu_apply_canonical(S, psi, dev), s.apply(psi), f"{p.model.name} n_up={p.n_up} two-pass")
        n_run += 1
    assert n_run >= 4


# (tile, grid, row order): order 1 deals segments of rows to the 8 XCDs
_TILE_CASES = ((1, 0, 0), (64, 7, 0), (128, 1024, 0), (256, 4096, 0), (512, 1, 0), (300, 0, 0),
               (512, 0, 1), (1, 0, 1), (128, 13, 1), (256, 2048, 1))


def test_spin_tile_tunings_bit_exact(dev):
    """Every short-row tile and grid of the spin kernel's sector queue gives
    the same vector bit for bit (each amplitude sums its terms in the same
    order however the rows are grouped), and it matches the oracle."""
    import torch
    cases = [p for p in _SPIN_CASES] + [I.heisenberg16()]
    n_run = 0
    for k, p in enumerate(cases):
        S = _ecut().Sectors.from_problem(p)
        if not S.info.kernel_flags & 4:
            continue
        s = O.Sector(p.model, p.n_up, p.n_dn)
        psi = I.psi(1300 + k, s.n)
        x = S.import_(torch.from_numpy(psi).to(dev))
        S.set_tuning(0, 0, 0, 0, 0)
        y0 = S.apply(x)
        for tile, grid, order in _TILE_CASES:
            S.set_tuning(grid, 0, order, 0, tile)
            y = S.apply(x)
            torch.cuda.synchronize()
            assert torch.equal(y, y0), f"{p.model.name} n_up={p.n_up} tile {tile} grid {grid} order {order}"
        S.set_tuning(0, 0, 0, 0, 64)
        _compare(_gpu_apply_canonical(S, psi, dev), s.apply(psi), f"{p.model.name} n_up={p.n_up} tile 64")
        n_run += 1
    assert n_run >= 4


def test_spin_tile_tunings_full_size(dev):
    """6x5 J1-J2 (155M amplitudes, 16 blocks): the tile and grid candidates of
    the autotuner give the default tuning's vector bit for bit."""
    import torch
    p = I.j1j2_6x5()
    S = _ecut().Sectors.from_problem(p)
    x = torch.from_numpy(I.psi(p.meta["seed"] + 5, S.dim)).to(dev)
    y0 = S.apply(x)
    y = torch.empty_like(x)
    for tile, grid, order in ((128, 1024, 0), (256, 4096, 0), (1, 0, 0), (512, 0, 1), (128, 512, 1), (512, 0, 1)):
        S.set_tuning(grid, 0, order, 0, tile)
        S.apply(x, out=y)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), (tile, grid, order)
    # the two-pass kernels: the same sums in the same order
    for rows, xcd in ((0, 8), (8, 8), (16, 1)):
        S.set_tuning(rows, xcd, 0, 2, 0)
        S.apply(x, out=y)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), ("two-pass", rows, xcd)
    # the generic row kernel walks the padded list of order 1 too
    S.set_tuning(0, 0, 1, 1, 0)
    S.apply(x, out=y)
    torch.cuda.synchronize()
    assert (torch.linalg.vector_norm(y - y0) / torch.linalg.vector_norm(y0)).item() <= RTOL
    del x, y, y0


def test_batch_mixed_kernels_bit_exact(dev):
    """A batch that mixes spin-kernel problems, generic-kernel problems, a
    spin problem tuned to the generic kernel, one on a padded XCD-dealt item
    list and a Hubbard problem on segment tiles runs each on its own kernel."""
    import torch
    ecut = _ecut()
    probs = [I.heisenberg16(), I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", 0b111), 10),
             _SPIN_CASES[-1], SMALL[3], I.heisenberg16(), I.hubbard12()]
    Ss = [ecut.Sectors.from_problem(p) for p in probs]
    assert Ss[0].info.kernel_flags & 4 and not Ss[1].info.kernel_flags & 4
    Ss[3].set_tuning(0, 0, 0, 1)
    Ss[4].set_tuning(0, 0, 1, 0, 64)     # padded XCD-dealt item list, small tile
    Ss[5].set_tuning(0, 8, 0, 5)         # Hubbard on segment tiles
    xs = [torch.from_numpy(I.psi(900 + k, S.dim)).to(dev) for k, S in enumerate(Ss)]
    alone = [S.apply(x) for S, x in zip(Ss, xs)]
    ys = [torch.empty_like(x) for x in xs]
    ecut.apply_batch(Ss, xs, ys)
    torch.cuda.synchronize()
    for k in range(len(Ss)):
        assert torch.equal(alone[k], ys[k]), f"batch differs for problem {k}"


def test_autotune_keeps_parity(dev, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("ECUT_TUNE_CACHE", str(tmp_path / "tune.json"))
    p = I.hubbard12()
    s = O.Sector(p.model, 6, 6)
    psi = I.psi(77, s.n)
    y_ref = s.apply(psi)
    S = _ecut().Sectors.from_problem(p)
    x = torch.from_numpy(psi).to(dev)
    best = S.autotune(x, torch.empty_like(x))
    assert (tmp_path / "tune.json").exists()
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"autotuned {best}")
    S2 = _ecut().Sectors.from_problem(p)
    assert S2.autotune(x, torch.empty_like(x)) == best      # served from the cache


def test_lanczos_heisenberg16_vs_oracle(dev):
    import torch
    p = I.heisenberg16()
    s = O.Sector(p.model, 8)
    e_ref = s.lanczos(I.psi(p.meta["seed"] + 1, s.n), 200, tol=1e-14)[0][-1]
    S = _ecut().Sectors.from_problem(p)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, s.n)).to(dev))
    e, st, _ = S.lanczos(v0, 100, fixed_steps=True)
    assert st["steps"] == 100
    assert abs(e - e_ref) <= 1e-10
    e2, st2, _ = S.lanczos(v0, 400, tol=1e-10)
    assert abs(e2 - e_ref) <= 1e-10 and st2["converged"] == 1
    for tile, order in ((1, 0), (64, 0), (64, 1)):
        # more, smaller work items, and the padded XCD-dealt list: the
        # per-item partial sums of the fused Lanczos epilogue follow the split;
        # a NaN workspace shows that every slot the solver reads is written
        # first and that padding writes none
        S.set_tuning(0, 0, order, 0, tile)
        ws = torch.full((S.lanczos_workspace(100),), float("nan"), dtype=torch.float64, device=dev)
        e3, st3, _ = S.lanczos(v0, 100, fixed_steps=True, workspace=ws)
        assert st3["steps"] == 100 and abs(e3 - e_ref) <= 1e-10, (tile, order, e3, e_ref)


@pytest.mark.parametrize("name", ["heisenberg16", "hubbard12"])
def test_lanczos_graph_replay_matches_eager(dev, name):
    """Three-term solves replayed from captured HIP graphs (one per ring phase)
    give the eagerly launched solve's energy and step count exactly: fixed-step
    runs (many replays of each graph) and runs to a tolerance, on the null
    stream (private capture stream) and on a stream of the caller's."""
    import torch
    p = I.WORKLOADS[name]()
    S = _ecut().Sectors.from_problem(p)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to(dev))
    side = torch.cuda.Stream()
    for kw in (dict(max_steps=150, fixed_steps=True), dict(max_steps=400, tol=1e-10)):
        e0, s0, _ = S.lanczos(v0, **kw)
        for stream in (None, side):
            e1, s1, _ = S.lanczos(v0, stream=stream, use_graph=True, **kw)
            torch.cuda.synchronize()
            assert e1 == e0 and s1["steps"] == s0["steps"], (kw, stream, e0, e1, s0["steps"], s1["steps"])
            # eager work between replays of the graphs of another solve
            y = S.apply(v0)
            torch.cuda.synchronize()
            del y


def test_lanczos_hubbard12_vs_oracle(dev):
    import torch
    p = I.hubbard12()
    s = O.Sector(p.model, 6, 6)
    e_ref = s.lanczos(I.psi(p.meta["seed"] + 1, s.n), 400, tol=1e-13)[0][-1]
    S = _ecut().Sectors.from_problem(p)
    v0 = torch.from_numpy(I.psi(p.meta["seed"] + 1, s.n)).to(dev)
    for variant in (0, 1, 3, 5):
        # a workspace full of NaN: every partial slot the solver reads must be written first
        S.set_tuning(0, 8, 0, variant)
        ws = torch.full((S.lanczos_workspace(200),), float("nan"), dtype=torch.float64, device=dev)
        e, st, _ = S.lanczos(v0, 200, fixed_steps=True, workspace=ws)
        assert st["steps"] == 200
        assert abs(e - e_ref) <= 1e-10, (variant, e, e_ref)


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", f"{name}_energy.json")) as f:
        return json.load(f)["energy"]


def test_lanczos_hubbard16_vs_golden(dev):
    """Full-size 16-site Hubbard chain (U=8): the 3-term solve to 1e-10 on
    the device reaches the oracle's stored ground energy (tests/golden,
    written by the oracle's own Lanczos on the full sparse H)."""
    import torch
    p = I.hubbard16()
    S = _ecut().Sectors.from_problem(p)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to(dev))
    e, st, _ = S.lanczos(v0, 400, tol=1e-10)
    assert st["converged"]
    assert abs(e - _golden("hubbard16")) <= 1e-10, (e, st)
    del v0
    torch.cuda.empty_cache()


def test_lanczos_j1j2_small_spin_kernel(dev):
    """Lanczos driven by the spin kernel on a 4x4 J1-J2 lattice against the
    oracle's energy on the same start vector."""
    import torch
    p = I.Problem(I.j1j2_lattice(4, 4, 1.0, 0.5), I.Cut("spatial", (1 << 8) - 1), 8)
    s = O.Sector(p.model, 8)
    e_ref = s.lanczos(I.psi(4321, s.n), 300, tol=1e-13)[0][-1]
    S = _ecut().Sectors.from_problem(p)
    assert S.info.kernel_flags & 4
    v0 = S.import_(torch.from_numpy(I.psi(4321, s.n)).to(dev))
    e, st, _ = S.lanczos(v0, 300, tol=1e-11)
    assert st["converged"] and abs(e - e_ref) <= 1e-10, (e, e_ref)


def test_lanczos_reorth_ground_state_vector(dev):
    import torch
    p = I.Problem(I.xxz_chain(14, 1.0, 0.6), I.Cut("spatial", I.left_mask_first(7)), 7)
    s = O.Sector(p.model, 7)
    H = s.dense()
    w, V = np.linalg.eigh(H)
    S = _ecut().Sectors.from_problem(p)
    v0 = torch.from_numpy(I.psi(9, s.n)).to(dev)
    e, st, gs = S.lanczos(v0, 60, tol=1e-11, reorth=True, max_restarts=4, want_gs=True)
    assert abs(e - w[0]) <= 1e-10
    g = S.export(gs).cpu().numpy()
    assert abs(abs(g @ V[:, 0]) - 1.0) <= 1e-8
    # H g = E g through the device H*psi
    hg = S.export(S.apply(gs)).cpu().numpy()
    assert np.linalg.norm(hg - e * g) <= 1e-6


def test_lanczos_reorth_unaligned_workspace_odd_dim(dev):
    """Full reorthogonalisation on a workspace that is 8- but not 16-byte
    aligned (the projection kernels then take their scalar-load path), on a
    sector of odd dimension (a one-element tail in the last chunk): the same
    energy, steps and ground state bit for bit as on an aligned workspace, and
    the oracle's energy."""
    import torch
    p = I.Problem(I.xxz_chain(15, 1.0, 0.6), I.Cut("spatial", I.left_mask_first(7)), 7)
    s = O.Sector(p.model, 7)
    assert s.n % 2 == 1
    ref = s.lanczos(I.psi(3, s.n), 600, tol=1e-14)[0][-1]
    S = _ecut().Sectors.from_problem(p)
    v0 = torch.from_numpy(I.psi(9, s.n)).to(dev)
    nws = S.lanczos_workspace(80, reorth=True, max_restarts=4, tol=1e-11)
    buf = torch.full((nws + 2,), float("nan"), dtype=torch.float64, device=dev)
    out = []
    for off in (0, 1):
        ws = buf[off:off + nws]
        assert (ws.data_ptr() % 16 == 0) == (off == 0)
        e, st, gs = S.lanczos(v0, 80, tol=1e-11, reorth=True, max_restarts=4, want_gs=True, workspace=ws)
        out.append((e, st["steps"], S.export(gs).cpu().numpy()))
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])
    assert abs(out[0][0] - ref) <= 1e-10


def test_lanczos_u0_hubbard16_closed_form(dev):
    """16-site chain at U=0 (the headline geometry): free-fermion energy."""
    import torch
    p = I.hubbard16(U=0.0)
    S = _ecut().Sectors.from_problem(p)
    eps = np.sort(-2.0 * np.cos(np.arange(1, 17) * np.pi / 17))
    e_ref = 2 * eps[:8].sum()
    assert e_ref == pytest.approx(-19.675902894918842, abs=1e-12)
    v0 = torch.empty(S.dim, dtype=torch.float64, device=dev).normal_(generator=torch.Generator(dev).manual_seed(1))
    e, st, _ = S.lanczos(v0, 400, tol=1e-11)
    assert abs(e - e_ref) <= 1e-10


def test_zero_start_vector_is_rejected(dev):
    import torch
    ecut = _ecut()
    S = ecut.Sectors.from_problem(I.heisenberg16())
    with pytest.raises(ecut.EcutError) as ei:
        S.lanczos(torch.zeros(S.dim, dtype=torch.float64, device=dev), 10, tol=1e-10)
    assert ei.value.status == ecut.ECUT_EINVAL


def test_not_converged_status(dev):
    import torch
    ecut = _ecut()
    S = ecut.Sectors.from_problem(I.heisenberg16())
    v0 = torch.from_numpy(I.psi(1, S.dim)).to(dev)
    e, st, _ = S.lanczos(v0, 3, tol=1e-12, allow_notconv=True)
    assert st["status"] == ecut.ECUT_ENOTCONV and st["steps"] == 3


def _serving_mix():
    reqs = []
    for n, d in [(12, 0.7), (14, 1.5), (10, 1.0), (16, 0.55)]:
        reqs.append(I.Problem(I.xxz_chain(n, 1.0, d), I.Cut("spatial", I.left_mask_first(n // 2)), n // 2))
    for L, U in [(8, 0.0), (8, 6.0), (10, 3.0), (6, 9.0)]:
        reqs.append(I.Problem(I.hubbard_chain(L, 1.0, U), I.Cut("updn"), L // 2, L // 2))
    return reqs


def test_server_batched_vs_alone_vs_oracle(dev):
    ecut = _ecut()
    reqs = _serving_mix()
    refs = []
    for p in reqs:
        s = O.Sector(p.model, p.n_up, p.n_dn)
        refs.append(s.lanczos(I.psi(3, s.n), 600, tol=1e-14)[0][-1])
    results = {}
    # alone_graph: one request at a time with graph replay; each request takes
    # the slot (and the host address) of the one before, so a replay must
    # never pick up the graphs of a retired request
    # lanes: two workers, the problems of at least 10,000 amplitudes (the
    # 16-site XXZ chain and the 10-site Hubbard chain) on their own stream
    for mode in ("alone", "mix", "mix_graph", "alone_graph", "lanes"):
        alone = mode.startswith("alone")
        # each new problem shape is tuned once per mode (one solve at a time:
        # the pick for the problem alone; several: kernels whose launches merge)
        srv = ecut.Server(2 << 30, max_active=(1 if alone else 0), max_steps=600, tol=1e-10,
                          sequential=alone, use_graph=mode.endswith("graph"), autotune=True,
                          large_dim=(10000 if mode == "lanes" else 0))
        print(f"[server] mode {mode}", flush=True)
        ids = [srv.submit(p, seed=1000 + k) for k, p in enumerate(reqs)]
        srv.drain()
        res = {r["req_id"]: r for r in srv.poll()}
        srv.close()
        results[mode] = [res[i] for i in ids]
    for k in range(len(reqs)):
        a, m = results["alone"][k], results["mix"][k]
        assert a["status"] == 0 and m["status"] == 0
        assert abs(a["energy"] - refs[k]) <= 1e-10, (k, a["energy"], refs[k])
        assert abs(m["energy"] - refs[k]) <= 1e-10, (k, m["energy"], refs[k])
        assert abs(a["energy"] - m["energy"]) <= 1e-10
        # the two modes may run different kernels (summation orders), so the
        # stopping step may move by one or two
        assert abs(a["steps"] - m["steps"]) <= 2
        # graph replay of the step changes nothing
        g = results["mix_graph"][k]
        assert g["status"] == 0 and g["energy"] == m["energy"] and g["steps"] == m["steps"]
        g = results["alone_graph"][k]
        assert g["status"] == 0 and g["energy"] == a["energy"] and g["steps"] == a["steps"]
        # two lanes: a large problem runs alone on its lane with the tuning
        # for a problem alone (the sequential run's vectors), the others
        # batch with the mix's tunings (the mix's vectors)
        g = results["lanes"][k]
        p = reqs[k]
        states = math.comb(p.model.n_sites, p.n_up) * (math.comb(p.model.n_sites, p.n_dn) if p.model.kind == "hubbard" else 1)
        same = a if states >= 10000 else m
        assert g["status"] == 0 and g["energy"] == same["energy"] and g["steps"] == same["steps"], k


def test_server_failed_build_is_reported(dev):
    """A request whose sectors cannot be built (checked only when the
    server's builder thread reaches it) finishes with the builder's error,
    and the requests around it are still solved, in order, to the oracle's
    energies; with graph replay and without."""
    ecut = _ecut()
    good = _serving_mix()[:3]
    bad = I.Problem(I.hubbard_chain(6, 1.0, 4.0), I.Cut("updn"), 7, 3)   # 7 > 6 sites
    refs = [O.Sector(p.model, p.n_up, p.n_dn).lanczos(I.psi(3, O.Sector(p.model, p.n_up, p.n_dn).n), 600,
                                                     tol=1e-14)[0][-1] for p in good]
    for use_graph in (False, True):
        srv = ecut.Server(1 << 30, max_steps=600, tol=1e-10, use_graph=use_graph)
        ids = [srv.submit(good[0], seed=1), srv.submit(bad, seed=2), srv.submit(good[1], seed=3),
               srv.submit(good[2], seed=4)]
        srv.drain()
        res = {r["req_id"]: r for r in srv.poll()}
        srv.close()
        assert sorted(res) == sorted(ids)
        assert res[ids[1]]["status"] == ecut.ECUT_EINVAL
        for k, i in zip((0, 1, 2), (ids[0], ids[2], ids[3])):
            assert res[i]["status"] == 0
            assert abs(res[i]["energy"] - refs[k]) <= 1e-10, (use_graph, k)


def test_server_budget_admission(dev):
    """A budget that holds one request at a time still serves them all
    (admission waits for memory); a request larger than the budget fails."""
    ecut = _ecut()
    small = I.Problem(I.xxz_chain(12, 1.0, 1.0), I.Cut("spatial", I.left_mask_first(6)), 6)
    big = I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", I.left_mask_first(10)), 10)
    one = 3 * 8 * math.comb(12, 6) + (1 << 16)
    srv = ecut.Server(int(one * 1.5), max_active=0, max_steps=400, tol=1e-10)
    ids = [srv.submit(small, seed=k) for k in range(3)] + [srv.submit(big, seed=9)]
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll()}
    srv.close()
    assert all(res[i]["status"] == 0 for i in ids[:3])
    assert res[ids[3]]["status"] == ecut.ECUT_ENOMEM
    e = [res[i]["energy"] for i in ids[:3]]
    assert max(e) - min(e) <= 1e-10


def test_server_two_lanes_share_the_budget(dev):
    """Two lanes over one small arena: a large request waits for the memory
    that the small lane's solves hold and is served once they retire; a
    large request over the budget and one whose sectors cannot be built fail
    on the large lane; every valid request matches the oracle."""
    ecut = _ecut()
    small = I.Problem(I.xxz_chain(12, 1.0, 0.9), I.Cut("spatial", I.left_mask_first(6)), 6)
    large = I.Problem(I.xxz_chain(16, 1.0, 1.1), I.Cut("spatial", I.left_mask_first(8)), 8)
    huge = I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", I.left_mask_first(10)), 10)
    bad = I.Problem(I.xxz_chain(40, 1.0, 1.0), I.Cut("spatial", I.left_mask_first(34)), 20)   # 34 > 32 sites
    refs = {}
    for name, p in (("small", small), ("large", large)):
        s = O.Sector(p.model, p.n_up, p.n_dn)
        refs[name] = s.lanczos(I.psi(3, s.n), 600, tol=1e-14)[0][-1]
    # room for one large solve, or for the four small ones, not for both (a
    # server solve's footprint is the three-term Lanczos workspace, in 256-byte
    # granules)
    def footprint(p):
        n = 8 * ecut.Sectors.from_problem(p, host_only=True).lanczos_workspace(600)
        return (n + 255) // 256 * 256
    f_small, f_large = footprint(small), footprint(large)
    budget = max(f_large, 4 * f_small) + 1024
    assert budget - 4 * f_small < f_large and budget < footprint(huge)
    srv = ecut.Server(budget, max_active=0, max_steps=600, tol=1e-10, large_dim=5000)
    ids = [srv.submit(small, seed=k) for k in range(4)]
    ids += [srv.submit(large, seed=7), srv.submit(huge, seed=8), srv.submit(bad, seed=9), srv.submit(large, seed=10)]
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll()}
    srv.close()
    assert sorted(res) == sorted(ids)
    for i in ids[:4]:
        assert res[i]["status"] == 0 and abs(res[i]["energy"] - refs["small"]) <= 1e-10
    for i in (ids[4], ids[7]):
        assert res[i]["status"] == 0 and abs(res[i]["energy"] - refs["large"]) <= 1e-10
    assert res[ids[5]]["status"] == ecut.ECUT_ENOMEM
    assert res[ids[6]]["status"] == ecut.ECUT_EUNSUPPORTED
    # FIFO inside the large lane: the second valid large request is admitted after the first
    assert res[ids[7]]["t_admit"] >= res[ids[4]]["t_admit"]


def test_server_two_lanes_memory_order(dev):
    """A large request waiting for arena space is not overtaken by small
    requests that arrived after it: with room for three small solves or the
    large one alone, the two small requests submitted after the large one are
    admitted only after it; every energy matches the oracle."""
    ecut = _ecut()
    small = I.Problem(I.xxz_chain(14, 1.0, 0.8), I.Cut("spatial", I.left_mask_first(7)), 7)
    large = I.Problem(I.xxz_chain(16, 1.0, 1.1), I.Cut("spatial", I.left_mask_first(8)), 8)
    refs = {}
    for name, p in (("small", small), ("large", large)):
        s = O.Sector(p.model, p.n_up, p.n_dn)
        refs[name] = s.lanczos(I.psi(3, s.n), 600, tol=1e-14)[0][-1]

    def footprint(p):
        n = 8 * ecut.Sectors.from_problem(p, host_only=True).lanczos_workspace(600)
        return (n + 255) // 256 * 256
    f_small, f_large = footprint(small), footprint(large)
    budget = f_large + 1024
    assert 3 * f_small <= budget < 4 * f_small and f_large + f_small > budget
    srv = ecut.Server(budget, max_active=0, max_steps=600, tol=1e-10, large_dim=5000)
    early = [srv.submit(small, seed=k) for k in range(3)]
    big = srv.submit(large, seed=7)
    late = [srv.submit(small, seed=10 + k) for k in range(2)]
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll()}
    srv.close()
    for i in early + late:
        assert res[i]["status"] == 0 and abs(res[i]["energy"] - refs["small"]) <= 1e-10
    assert res[big]["status"] == 0 and abs(res[big]["energy"] - refs["large"]) <= 1e-10
    # the large solve never shares the arena with a small one, and the late
    # small requests come after it
    for i in late:
        assert res[i]["t_admit"] >= res[big]["t_done"] - 1e-9, (res[i], res[big])
    for i in early:
        assert res[i]["t_done"] <= res[big]["t_admit"] + 1e-9


def test_caller_allocator_backs_sector_tables(dev):
    """ecut_set_allocator: sector tables taken from torch's caching allocator
    give the same H*psi bit for bit; a server builds and frees its requests'
    tables through the callbacks from its own threads; every block goes back
    through the pair that made it; a block that is not 256-byte aligned is
    refused and handed back."""
    import torch
    E = _ecut()
    ta, tf = E.torch_allocator()
    live, log = {}, []

    def alloc(n, d):
        ptr = ta(n, d)
        live[ptr] = n
        log.append("a")
        return ptr

    def free(ptr, n, d):
        assert live.pop(ptr) == n
        log.append("f")
        tf(ptr, n, d)

    probs = [I.Problem(I.xxz_chain(12, 1.0, 0.7), I.Cut("spatial", I.left_mask_first(6)), 6),
             I.Problem(I.hubbard_chain(8, 1.0, 6.0), I.Cut("updn"), 4, 4)]
    refs = []
    for p in probs:
        S = E.Sectors.from_problem(p)
        x = torch.from_numpy(I.psi(5, S.dim)).to(dev)
        refs.append((x, S.apply(x).cpu()))
        S.close()
    E.set_allocator(alloc, free)
    try:
        for p, (x, yref) in zip(probs, refs):
            S = E.Sectors.from_problem(p)
            assert len(live) == 1
            y = S.apply(x).cpu()
            S.close()
            assert torch.equal(y, yref)
        assert not live
        srv = E.Server(1 << 30, max_steps=300, tol=1e-10)
        ids = [srv.submit(p, seed=7 + k) for k, p in enumerate(probs)]
        srv.drain()
        res = srv.poll()
        srv.close()
        assert sorted(r["req_id"] for r in res) == sorted(ids)
        assert all(r["status"] == 0 for r in res)
        assert not live and log.count("a") == log.count("f") == 4
        E.set_allocator(lambda n, d: ta(n + 256, d) + 8, lambda ptr, n, d: tf(ptr - 8, n, d))
        with pytest.raises(E.EcutError) as err:
            E.Sectors.from_problem(probs[0])
        assert err.value.status == E.ECUT_EINVAL
    finally:
        E.set_allocator()
    S = E.Sectors.from_problem(probs[0])
    y = S.apply(refs[0][0]).cpu()
    S.close()
    assert torch.equal(y, refs[0][1])


def test_lanczos_j1j2_6x5_vs_golden(dev):
    """6x5 J1-J2 lattice (155,117,520 states, 16 blocks), autotuned spin
    kernel: the three-term solve to 1e-10 reaches the oracle's stored ground
    energy (tests/golden, the oracle's own Lanczos on the full sparse H)."""
    import torch
    p = I.j1j2_6x5()
    S = _ecut().Sectors.from_problem(p)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to(dev))
    S.autotune(v0, torch.empty_like(v0))
    e, st, _ = S.lanczos(v0, 600, tol=1e-10)
    assert st["converged"]
    assert abs(e - _golden("j1j2_6x5")) <= 1e-10, (e, st)
    del v0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("large_dim", [0, 1 << 22])
def test_server_mix_vs_oracle_per_request(dev, large_dim):
    """The first 48 requests of the 256-request serving mix (XXZ chains of
    12-24 sites and Hubbard chains of 8-14 sites), batched with continuous
    admission, on one worker and on two (the 14-site Hubbard chains on their
    own lane): every energy within 1e-10 of the oracle's energy for that
    request (tests/golden/serving_2026_energies.json)."""
    import json
    import os
    ecut = _ecut()
    with open(os.path.join(os.path.dirname(__file__), "golden", "serving_2026_energies.json")) as f:
        ref = [e["energy"] for e in json.load(f)["energies"]]
    reqs = I.serving_requests(256, seed=2026)[:48]
    srv = ecut.Server(24 << 30, max_active=32, max_steps=600, tol=1e-10, autotune=True, large_dim=large_dim)
    ids = [srv.submit(p, seed=p.meta["seed"]) for p in reqs]
    srv.drain()
    res = {r["req_id"]: r for r in srv.poll(64)}
    srv.close()
    err = [abs(res[i]["energy"] - ref[k]) for k, i in enumerate(ids)]
    assert all(res[i]["status"] == 0 for i in ids)
    assert max(err) <= 1e-10, (int(np.argmax(err)), max(err))


def test_hubbard_batch_one_launch_bit_exact(dev):
    """A Hubbard-heavy batch on the two-pass kernels (chains of 6 to 12 sites
    with random U, random long-range hoppings with fermion signs, odd row
    lengths) runs in one merged launch per pass: every output equals the
    problem's own application bit for bit and the oracle's vector; spin
    problems in the same batch keep their own queue."""
    import torch
    E = _ecut()
    rng = np.random.default_rng(4242)
    probs = []
    for L in (6, 8, 10, 12, 8, 10):
        probs.append(I.Problem(I.hubbard_chain(L, 1.0, float(rng.uniform(0, 10))), I.Cut("updn"), L // 2, L // 2))
    probs.append(I.Problem(I.random_hubbard_model(np.random.default_rng(5), 9, n_bonds=14), I.Cut("updn"), 4, 5))
    probs.append(I.Problem(I.hubbard_chain(7, 1.0, 2.0), I.Cut("updn"), 3, 2))
    probs.append(I.heisenberg16())
    probs.append(I.Problem(I.xxz_chain(12, 1.0, 0.8), I.Cut("spatial", I.left_mask_first(6)), 6))
    Ss = [E.Sectors.from_problem(p) for p in probs]
    for k, S in enumerate(Ss):
        if probs[k].model.kind == "hubbard":
            S.set_tuning(0, 8, 1, 6, 2 if k % 2 else 4)
    psis = [I.psi(2100 + k, S.dim) for k, S in enumerate(Ss)]
    xs = [S.import_(torch.from_numpy(x).to(dev)) for S, x in zip(Ss, psis)]
    alone = [S.apply(x) for S, x in zip(Ss, xs)]
    ys = [torch.empty_like(x) for x in xs]
    E.apply_batch(Ss, xs, ys)
    torch.cuda.synchronize()
    for k, (p, S) in enumerate(zip(probs, Ss)):
        assert torch.equal(alone[k], ys[k]), f"batch differs for problem {k} ({p.model.name})"
        s = O.Sector(p.model, p.n_up, p.n_dn)
        _compare(S.export(ys[k]).cpu().numpy(), s.apply(psis[k]), f"batched {p.model.name}")


def _ent_compare(got, ref, what, lam_tol):
    nb = len(ref["lam"])
    assert len(got["lam"]) == nb
    for q in range(nb):
        a, b = got["lam"][q], ref["lam"][q]
        assert a.shape == b.shape, (what, q)
        assert np.max(np.abs(a - b), initial=0.0) <= lam_tol, (what, q, np.max(np.abs(a - b)))
    np.testing.assert_allclose(got["w_q"], ref["w_q"], atol=lam_tol * 10, err_msg=what)
    assert abs(got["entropy"] - ref["entropy"]) <= lam_tol * 1e3, what
    assert abs(got["weight_ipr"] - ref["weight_ipr"]) <= lam_tol * 1e3 * ref["weight_ipr"], what


@pytest.mark.parametrize("name", ["heisenberg16", "hubbard12"])
def test_entanglement_spectrum_vs_oracle(dev, name):
    """The oracle's ground state (ARPACK on the oracle's H), imported into
    the bipartite layout: the device spectrum of rho_L per block (Gram matrix
    + symmetric eigensolver) against numpy's singular values of the oracle's
    own blocks (|d lambda| <= 1e-13: the Gram matrix carries an absolute
    error of about eps * lambda_max), W_q, the entropy, the weight IPR,
    N_eff of the sector Schmidt ranks and W_P over (up to) 3 parts."""
    import torch
    p = I.WORKLOADS[name]()
    s = O.Sector(p.model, p.n_up, p.n_dn)
    e0, g = O.ground_state(s, I.psi(p.meta["seed"] + 1, s.n))
    S = _ecut().Sectors.from_problem(p)
    nb = S.info.n_blocks
    parts = np.arange(nb) % 3
    ref = O.entanglement(s, g, p.cut.kind, p.cut.left_mask, parts=parts, cutoff=1e-10)
    x = S.import_(torch.from_numpy(g).to(dev))
    got = S.entanglement(x, n_parts=int(parts.max()) + 1, part_of_block=parts, cutoff=1e-10)
    _ent_compare(got, ref, name, 1e-13)
    assert abs(got["n_eff"] - ref["n_eff"]) <= 1e-12
    np.testing.assert_allclose(got["w_p"], ref["w_p"], atol=1e-12)
    assert abs(got["w_q"].sum() - 1.0) <= 1e-12
    # the same state at another norm gives the same spectrum
    got2 = S.entanglement(3.0 * x, n_parts=1, cutoff=1e-10)
    _ent_compare(got2, ref, name + " x3", 1e-13)


def test_entanglement_of_device_ground_state(dev):
    """End to end: the device's own ground state (Lanczos with full
    reorthogonalisation to a residual of 1e-8, 14-site XXZ chain, spatial
    cut 7|7) against the oracle's: equal up to the vector's accuracy
    (|d lambda| <= 1e-7, about residual / spectral gap)."""
    import torch
    p = I.Problem(I.xxz_chain(14, 1.0, 0.6), I.Cut("spatial", I.left_mask_first(7)), 7)
    s = O.Sector(p.model, p.n_up)
    e0, g = O.ground_state(s, I.psi(11, s.n))
    ref = O.entanglement(s, g, "spatial", p.cut.left_mask)
    S = _ecut().Sectors.from_problem(p)
    v0 = torch.from_numpy(I.psi(12, S.dim)).to(dev)
    e, st, gs = S.lanczos(v0, 80, tol=1e-12, reorth=True, max_restarts=6, want_gs=True)
    assert abs(e - e0) <= 1e-10
    got = S.entanglement(gs, cutoff=1e-14)
    _ent_compare(got, ref, "device ground state", 1e-7)


def test_entanglement_rejects_bad_arguments(dev):
    import torch
    E = _ecut()
    S = E.Sectors.from_problem(I.heisenberg16())
    with pytest.raises(E.EcutError) as err:
        S.entanglement(torch.zeros(S.dim, dtype=torch.float64, device=dev))
    assert err.value.status == E.ECUT_EINVAL
    with pytest.raises(E.EcutError) as err:
        S.entanglement(torch.ones(S.dim, dtype=torch.float64, device=dev), n_parts=2,
                       part_of_block=np.full(S.info.n_blocks, 2))
    assert err.value.status == E.ECUT_EINVAL


_CDAG_CASES = [(I.hubbard_chain(8, 1.0, 3.0), 4, 3), (I.hubbard_chain(7, 1.0, 2.0), 2, 4),
               (I.random_hubbard_model(np.random.default_rng(61), 9, n_bonds=14), 4, 4),
               (I.hubbard_chain(22, 1.0, 3.0), 2, 1)]   # beyond the up/down kernels' tables: colex columns


@pytest.mark.parametrize("k", range(len(_CDAG_CASES)))
def test_apply_cdag_vs_oracle(dev, k):
    """c+ and c of every site and spin between Hubbard sectors equal the
    oracle's full-basis operator bit for bit (a signed permutation), in
    class-major and in colex column layouts."""
    import torch
    E = _ecut()
    m, nu, nd = _CDAG_CASES[k]
    L = m.n_sites
    S0 = E.Sectors.from_problem(I.Problem(m, I.Cut("updn"), nu, nd))
    s0 = O.Sector(m, nu, nd)
    x = I.psi(2400 + k, s0.n)
    xb = S0.import_(torch.from_numpy(x).to(dev))
    sites = range(L) if L <= 9 else (0, 5, L - 1)
    for spin in (0, 1):
        for dagger in (True, False):
            nu1, nd1 = nu + (spin == 0) * (1 if dagger else -1), nd + (spin == 1) * (1 if dagger else -1)
            if not (0 <= nu1 <= L and 0 <= nd1 <= L):
                continue
            S1 = E.Sectors.from_problem(I.Problem(m, I.Cut("updn"), nu1, nd1))
            s1 = O.Sector(m, nu1, nd1)
            for site in sites:
                y = S1.export(E.apply_cdag(S0, S1, site, spin, dagger, xb)).cpu().numpy()
                ref = O.apply_cdag(s0, s1, site, spin, dagger, x)
                assert np.array_equal(y, ref), (m.name, spin, dagger, site)
            S1.close()
    with pytest.raises(E.EcutError) as err:   # a destination that does not match the operator
        E.apply_cdag(S0, S0, 0, 0, True, xb)
    assert err.value.status == E.ECUT_EINVAL


@pytest.mark.parametrize("site,spin,dagger", [(3, 0, True), (0, 1, False), (5, 1, True)])
def test_green_function_vs_oracle(dev, site, spin, dagger):
    """12-site Hubbard chain (U=4, half filling): from the oracle's ground
    state, c+ psi0 (or c psi0) on the device, 60 Lanczos steps of the target
    sector's H and the continued fraction, against the oracle's operator,
    its own Lanczos coefficients and continued fraction on the same start
    vector: weight to 1e-13, the first 10 coefficients to 1e-10 (two
    three-term recurrences in different summation orders part once the
    extreme Ritz values converge and orthogonality is lost, after about a
    dozen steps here), and G(w) on a grid at eta = 0.5, where both continued
    fractions have converged, to 1e-6 of its largest value."""
    import torch
    E = _ecut()
    p = I.hubbard12()
    s0 = O.Sector(p.model, 6, 6)
    e0, g = O.ground_state(s0, I.psi(1, s0.n))
    d = 1 if dagger else -1
    nu1, nd1 = 6 + (spin == 0) * d, 6 + (spin == 1) * d
    s1 = O.Sector(p.model, nu1, nd1)
    phi = O.apply_cdag(s0, s1, site, spin, dagger, g)
    w_ref = phi @ phi
    _, a_ref, b_ref = s1.lanczos(phi, 60)
    omega = np.linspace(-10, 10, 201)
    G_ref = O.continued_fraction(a_ref, b_ref, w_ref, e0, dagger, omega, 0.5)
    S0 = E.Sectors.from_problem(p)
    S1 = E.Sectors.from_problem(I.Problem(p.model, I.Cut("updn"), nu1, nd1))
    gb = S0.import_(torch.from_numpy(g).to(dev))
    G, a, b, w = E.green_function(S0, gb, e0, S1, site, spin, dagger, 60, omega, 0.5)
    assert abs(w - w_ref) <= 1e-13 * max(w_ref, 1.0)
    assert len(a) == 60
    np.testing.assert_allclose(a[:10], a_ref[:10], atol=1e-10)
    np.testing.assert_allclose(b[:10], b_ref[:10], atol=1e-10)
    assert np.max(np.abs(G - G_ref)) <= 1e-6 * np.max(np.abs(G_ref)), np.max(np.abs(G - G_ref))
    # the library's continued fraction on the oracle's coefficients is the oracle's
    np.testing.assert_allclose(E.continued_fraction(a_ref, b_ref, w_ref, e0, dagger, omega, 0.5), G_ref, atol=1e-13)


# ---------------------------------------------------------------- spatial-cut Hubbard (fermionic cross terms, V)

def _spatial_hubbard_cases():
    rng = np.random.default_rng(2605)
    out = []
    for n, nu, nd in ((2, 1, 1), (4, 2, 1), (5, 2, 3), (6, 3, 3), (7, 4, 2), (8, 3, 5), (9, 4, 4), (10, 5, 5)):
        m = I.random_extended_hubbard_model(rng, n)
        out.append((m, int(rng.integers(1, (1 << n) - 1)), nu, nd))
    out.append((I.hubbard_chain(6, V=1.0), (1 << 6) - 1, 3, 2))   # everything on the left
    out.append((I.hubbard_chain(6, V=1.0), 0, 2, 3))              # everything on the right
    out.append((I.hubbard_chain(8, 1.0, 4.0, periodic=True, V=1.5), 0b10101010, 4, 4))
    out.append((I.hubbard_chain(8, V=1.0), 0b11110000, 0, 4))     # one spin species empty
    return out


@pytest.mark.parametrize("k", range(len(_spatial_hubbard_cases())))
def test_spatial_hubbard_apply_vs_oracle(dev, k):
    """Hubbard models with bond interactions V on random (also long-range)
    bonds, cut by random site masks: H*psi in the bipartite layout, with the
    fermion signs of hops across the cut, against the oracle's occupation-
    basis H (canonical order, through the signed layout map)."""
    m, mask, nu, nd = _spatial_hubbard_cases()[k]
    S = _ecut().Sectors(m, I.Cut("spatial", mask), nu, nd)
    s = O.Sector(m, nu, nd)
    psi = I.psi(2700 + k, s.n)
    y_ref = s.apply(psi)
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{m.name} mask {mask:#x}")
    # the two-pass row kernels (signed source-column tables), every item shape
    assert S.info.kernel_flags & 64
    for rows, xcd in ((0, 8), (4, 1), (16, 8), (32, 1)):
        S.set_tuning(rows, xcd, 0, 2, 0)
        _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{m.name} mask {mask:#x} two-pass {rows},{xcd}")
    S.set_tuning(0, 0, 0, 0, 0)   # and back to the row kernel
    _compare(_gpu_apply_canonical(S, psi, dev), y_ref, f"{m.name} mask {mask:#x} row kernel again")


def test_spatial_hubbard14_full_vector_vs_oracle(dev):
    """The paper's spatial-cut Hubbard ED size: 14-site chain, t=1, U=4,
    V=1, N_up=N_dn=7, cut in the middle (11,778,624 amplitudes in 64
    blocks): the whole H*psi against the oracle's; Hermiticity on the
    device; cut invariance (for V=0 the spatial and up/down cuts give the
    same canonical H*psi)."""
    import time
    import torch
    E = _ecut()
    m = I.hubbard_chain(14, 1.0, 4.0, V=1.0)
    S = E.Sectors(m, I.Cut("spatial", I.left_mask_first(7)), 7, 7)
    assert S.info.n_blocks == 64
    s = O.Sector(m, 7, 7)
    psi = I.psi(2750, s.n)
    t0 = time.time()
    y_ref = s.apply(psi, use_csr=False)
    print(f"[full] oracle apply {time.time() - t0:.1f} s", flush=True)
    _compare_full(_gpu_apply_canonical(S, psi, dev), y_ref, "spatial hubbard14 V=1")
    S.set_tuning(8, 8, 0, 2, 0)
    _compare_full(_gpu_apply_canonical(S, psi, dev), y_ref, "spatial hubbard14 V=1, two-pass")
    x = torch.from_numpy(psi).to(dev)
    print("[full] spatial hubbard14 autotuned", S.autotune(S.import_(x), torch.empty_like(x)), flush=True)
    _compare_full(_gpu_apply_canonical(S, psi, dev), y_ref, "spatial hubbard14 V=1, autotuned")
    xb = S.import_(torch.from_numpy(psi).to(dev))
    pb = S.import_(torch.from_numpy(I.psi(2751, s.n)).to(dev))
    lhs = torch.dot(pb, S.apply(xb)).item()
    rhs = torch.dot(S.apply(pb), xb).item()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    m0 = I.hubbard_chain(14, 1.0, 4.0)
    a = _gpu_apply_canonical(E.Sectors(m0, I.Cut("spatial", I.left_mask_first(7)), 7, 7), psi, dev)
    b = _gpu_apply_canonical(E.Sectors(m0, I.Cut("updn"), 7, 7), psi, dev)
    _compare_full(a, b, "spatial vs up/down cut, V=0")


def test_spatial_hubbard_lanczos_and_entanglement_vs_oracle(dev):
    """10-site extended Hubbard chain (t=1, U=4, V=1.5, 5+5 particles), cut
    5|5: the device Lanczos ground energy against ARPACK on the oracle's H,
    and the entanglement spectrum of the oracle's ground state across the
    fermionic mode partition (blocks (N_up_L, N_dn_L)) against numpy's
    singular values of the oracle's signed blocks."""
    import torch
    m = I.hubbard_chain(10, 1.0, 4.0, V=1.5)
    S = _ecut().Sectors(m, I.Cut("spatial", I.left_mask_first(5)), 5, 5)
    s = O.Sector(m, 5, 5)
    e0, g = O.ground_state(s, I.psi(2760, s.n))
    v0 = torch.from_numpy(I.psi(2761, S.dim)).to(dev)
    e, st, _ = S.lanczos(v0, 300, tol=1e-12)
    assert abs(e - e0) <= 1e-10 * abs(e0), (e, e0)
    S.set_tuning(8, 8, 0, 2, 0)   # the two-pass row kernels, with the Lanczos partials of their items
    e2, st2, _ = S.lanczos(v0, 300, tol=1e-12)
    assert abs(e2 - e0) <= 1e-10 * abs(e0), (e2, e0)
    S.set_tuning(0, 0, 0, 0, 0)
    ref = O.entanglement(s, g, "spatial", I.left_mask_first(5), cutoff=1e-10)
    got = S.entanglement(S.import_(torch.from_numpy(g).to(dev)), cutoff=1e-10)
    _ent_compare(got, ref, "spatial hubbard10", 1e-13)
    assert abs(got["n_eff"] - ref["n_eff"]) <= 1e-12


def test_lanczos_hubbard14_spatial_vs_golden(dev):
    """The paper's spatial-cut ED benchmark (14-site extended Hubbard chain,
    V=1, cut 7|7) on the autotuned kernel: three-term Lanczos to 1e-10
    against the oracle's energy (tests/golden, written from the oracle's CSR
    to 1e-14)."""
    import json
    import os
    import torch
    p = I.hubbard14_spatial()
    with open(os.path.join(os.path.dirname(__file__), "golden", "hubbard14_spatial_energy.json")) as f:
        ref = json.load(f)["energy"]
    S = _ecut().Sectors.from_problem(p)
    x = torch.from_numpy(I.psi(p.meta["seed"], S.dim)).to(dev)
    print("[full] hubbard14_spatial autotuned", S.autotune(S.import_(x), torch.empty_like(x)), flush=True)
    v0 = S.import_(torch.from_numpy(I.psi(p.meta["seed"] + 1, S.dim)).to(dev))
    e, st, _ = S.lanczos(v0, 600, tol=1e-10)
    assert st["converged"] and abs(e - ref) <= 1e-10, (e, ref)


def test_batch_with_two_pass_row_problems_bit_exact(dev):
    """A batch of spatial-cut Hubbard problems on the two-pass row kernels
    (and one on the row kernel), spin problems on the two-pass and on the
    one-pass kernels, and up/down Hubbard problems in the merged launches:
    every output equals the problem's own application bit for bit, and the
    oracle's vector; the same through the no-allocation entry point."""
    import torch
    E = _ecut()
    rng = np.random.default_rng(77)
    probs = [I.Problem(I.random_extended_hubbard_model(rng, 8), I.Cut("spatial", 0b10110101), 4, 3),
             I.Problem(I.hubbard_chain(10, 1.0, 3.0, V=0.7), I.Cut("spatial", I.left_mask_first(5)), 5, 5),
             I.Problem(I.hubbard_chain(8, 1.0, 2.0, V=1.2), I.Cut("spatial", I.left_mask_first(4)), 4, 4),
             I.heisenberg16(),
             I.Problem(I.xxz_chain(14, 1.0, 0.8), I.Cut("spatial", I.left_mask_first(7)), 7),
             I.Problem(I.hubbard_chain(8, 1.0, 4.0), I.Cut("updn"), 4, 4)]
    tunings = [(8, 8, 0, 2, 0), (0, 1, 0, 2, 0), (0, 0, 0, 0, 0), (4, 8, 0, 2, 0), (0, 0, 0, 0, 0), (0, 8, 1, 6, 2)]
    Ss = [E.Sectors.from_problem(p) for p in probs]
    for S, t in zip(Ss, tunings):
        S.set_tuning(*t)
    psis = [I.psi(2900 + k, S.dim) for k, S in enumerate(Ss)]
    xs = [S.import_(torch.from_numpy(x).to(dev)) for S, x in zip(Ss, psis)]
    alone = [S.apply(x) for S, x in zip(Ss, xs)]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    ys2 = [torch.full_like(x, float("nan")) for x in xs]
    E.apply_batch(Ss, xs, ys)
    E.apply_batch(Ss, xs, ys2, noalloc=True)
    torch.cuda.synchronize()
    for k, (p, S) in enumerate(zip(probs, Ss)):
        assert torch.equal(alone[k], ys[k]), f"batch differs for problem {k} ({p.model.name})"
        assert torch.equal(alone[k], ys2[k]), f"no-allocation batch differs for problem {k} ({p.model.name})"
        s = O.Sector(p.model, p.n_up, p.n_dn)
        _compare(S.export(ys[k]).cpu().numpy(), s.apply(psis[k]), f"batched {p.model.name}")
