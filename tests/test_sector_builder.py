"""Host-side tests of libecut (no GPU): the library loads and exports every
declared symbol, the sector builder's bases, blocks and canonical->bipartite
positions equal the oracle's enumeration bit for bit, and argument errors
come back as status codes."""
import math
import re
import os

import numpy as np
import pytest

import oracle as O
from paper_2605_07621_amd import inputs as I
from paper_2605_07621_amd import ecut as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ecut.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(ecut_[A-Za-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 18
    L = E.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    bound = {n for n, _, _ in E.SYMBOLS}
    assert declared == bound
    assert b"gfx950" in L.ecut_version()


def test_set_allocator_argument_checks():
    """ecut_set_allocator takes both callbacks or neither (no device work)."""
    L = E.lib()
    assert L.ecut_set_allocator(E.ALLOC_FN(lambda n, d, u: None), E.FREE_FN(), None) == E.ECUT_EINVAL
    assert b"both" in L.ecut_last_error()
    assert L.ecut_set_allocator(E.ALLOC_FN(), E.FREE_FN(lambda p, n, d, u: None), None) == E.ECUT_EINVAL
    assert L.ecut_set_allocator(E.ALLOC_FN(), E.FREE_FN(), None) == E.ECUT_OK
    with pytest.raises(ValueError):
        E.set_allocator(lambda n, d: 0, None)
    E.set_allocator(lambda n, d: 0, lambda p, n, d: None)
    E.set_allocator()


def _oracle_blocks_and_pos(p):
    s = O.Sector(p.model, p.n_up, p.n_dn)
    pos, blocks = s.bipartite(p.cut.kind, p.cut.left_mask)
    return s, pos, blocks


CASES = [
    I.heisenberg16(),
    I.hubbard12(),
    I.Problem(I.xxz_chain(10, 1.0, 0.7), I.Cut("spatial", 0b1000110101), 5),
    I.Problem(I.xxz_chain(9, 1.0, 1.3), I.Cut("spatial", 0b1), 3),
    I.Problem(I.xxz_chain(7, 1.0, 1.0), I.Cut("spatial", 0), 3),          # empty left part
    I.Problem(I.xxz_chain(7, 1.0, 1.0), I.Cut("spatial", 0b1111111), 2),  # empty right part
    I.Problem(I.j1j2_lattice(4, 3), I.Cut("spatial", I.left_mask_first(6)), 6),
    I.Problem(I.hubbard_chain(6, 1.0, 3.0), I.Cut("updn"), 2, 4),
    I.Problem(I.hubbard_chain(5, 1.0, 3.0), I.Cut("updn"), 0, 5),
    # the two headline sizes: 165,636,900 and 155,117,520 positions, every one
    # checked against the oracle's own enumeration
    I.hubbard16(),
    I.j1j2_6x5(),
]


def _class_major(words, n_sites):
    """Column order of the down words under the Hubbard up/down kernels:
    by popcount of the high half (sites n/2..n-1), then the high half, then
    the low half (the class-major order, so every class is contiguous).
    Returns (words in column order, column of the word of canonical rank r)."""
    h = n_sites // 2
    w = [int(v) for v in words]
    order = sorted(range(len(w)), key=lambda r: (bin(w[r] >> h).count("1"), w[r] >> h, w[r] & ((1 << h) - 1)))
    col = np.empty(len(w), dtype=np.int64)
    col[order] = np.arange(len(w))
    return np.asarray([w[r] for r in order], dtype=np.uint64), col


@pytest.mark.parametrize("p", CASES, ids=lambda p: f"{p.model.name}-{p.cut.kind}-{p.n_up}-{p.n_dn}")
def test_blocks_words_positions_bit_exact(p):
    S = E.Sectors.from_problem(p, host_only=True)
    s, pos, oblocks = _oracle_blocks_and_pos(p)
    blocks = S.blocks()
    assert S.dim == s.n
    assert blocks.shape[0] == oblocks.shape[0]
    np.testing.assert_array_equal(blocks[:, 0], oblocks[:, 0])   # q_l
    np.testing.assert_array_equal(blocks[:, 2], oblocks[:, 1])   # d_L
    np.testing.assert_array_equal(blocks[:, 3], oblocks[:, 2])   # d_R
    np.testing.assert_array_equal(blocks[:, 4], oblocks[:, 3])   # offsets
    class_major = p.cut.kind == "updn" and S.info.kernel == 1
    if class_major:
        # the oracle's positions with the down index replaced by its column
        dR = int(blocks[0, 3])
        _, col = _class_major(O.enumerate_bruteforce(p.model.n_sites, p.n_dn), p.model.n_sites)
        pos = (pos // dR) * dR + col[pos % dR]
    np.testing.assert_array_equal(S.canonical_positions(), pos)
    for b in range(blocks.shape[0]):
        lw, rw = S.words(b)
        if p.cut.kind == "spatial":
            n_left = bin(p.cut.left_mask).count("1")
            n_right = p.model.n_sites - n_left
        else:
            n_left = n_right = p.model.n_sites
        ql, qr = int(blocks[b, 0]), int(blocks[b, 1])
        want_r = O.enumerate_bruteforce(n_right, qr) if n_right else np.asarray([0], dtype=np.uint64)
        if class_major:
            want_r = _class_major(want_r, p.model.n_sites)[0]
        np.testing.assert_array_equal(lw.astype(np.uint64), O.enumerate_bruteforce(n_left, ql) if n_left else [0])
        np.testing.assert_array_equal(rw.astype(np.uint64), want_r)


def test_workload_block_structure():
    S = E.Sectors.from_problem(I.heisenberg16(), host_only=True)
    b = S.blocks()
    assert list(b[:, 2] * b[:, 3]) == [math.comb(8, k) ** 2 for k in range(9)]
    S4 = E.Sectors.from_problem(I.j1j2_6x5(), host_only=True)
    b4 = S4.blocks()
    assert b4.shape[0] == 16 and S4.dim == 155117520
    assert list(b4[:, 2] * b4[:, 3]) == [math.comb(15, k) ** 2 for k in range(16)]
    # a straight cut between x=2 and x=3 of the 6x5 lattice crosses 5 J1 and 8 J2 bonds
    assert S4.info.n_cut_bonds == 13 and S4.info.n_cross_offdiag == 26 and S4.info.n_cross_diag == 13
    S5 = E.Sectors.from_problem(I.hubbard14_spatial(), host_only=True)
    assert S5.dim == 3432 ** 2 and S5.info.n_blocks == 64 and S5.info.kernel == 2 and S5.info.kernel_flags == 64
    assert sorted(map(tuple, S5.labels()[:, :2].tolist())) == [(a, b) for a in range(8) for b in range(8)]
    S3 = E.Sectors.from_problem(I.hubbard16(), host_only=True)
    assert S3.dim == 165636900 and S3.info.kernel == 1 and S3.info.kernel_flags == 1 | 2 | 8 | 16 | 32
    assert S3.info.n_eff == pytest.approx(1.0)


def test_spin_kernel_eligibility():
    # the ranking-table spin kernel needs both parts <= 16 sites, row tiles
    # that fit its work group and <= 64 flip-flop terms inside the right part
    for p in (I.heisenberg16(), I.j1j2_6x5(), I.Problem(I.xxz_chain(24, 1.0, 0.7), I.Cut("spatial", (1 << 12) - 1), 12)):
        S = E.Sectors.from_problem(p, host_only=True)
        assert S.info.kernel == 2 and S.info.kernel_flags == 4 | 64, p.model.name
    wide = I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", 0b111), 10)   # right part: 17 sites
    assert E.Sectors.from_problem(wide, host_only=True).info.kernel_flags == 0
    dense = I.Problem(I.random_spin_model(np.random.default_rng(3), 14, n_bonds=91), I.Cut("spatial", 0b1), 7)
    assert E.Sectors.from_problem(dense, host_only=True).info.kernel_flags == 0   # 78 flip-flop terms on the right


def test_n_eff_is_block_participation_number():
    S = E.Sectors.from_problem(I.heisenberg16(), host_only=True)
    b = S.blocks()
    w = (b[:, 2] * b[:, 3]) / S.dim
    assert S.info.n_eff == pytest.approx(1.0 / np.sum(w * w), rel=1e-12)


def _status(fn):
    try:
        fn()
    except E.EcutError as e:
        return e.status
    return E.ECUT_OK


def test_error_paths():
    m = I.heisenberg_chain(6)
    assert _status(lambda: E.Sectors(m, I.Cut("updn"), 3, host_only=True)) == E.ECUT_EINVAL
    assert _status(lambda: E.Sectors(m, I.Cut("spatial", 0b111), 7, host_only=True)) == E.ECUT_EINVAL
    assert _status(lambda: E.Sectors(m, I.Cut("spatial", 1 << 9), 3, host_only=True)) == E.ECUT_EINVAL
    h = I.hubbard_chain(6)
    hv = I.hubbard_chain(6, V=1.0)
    assert _status(lambda: E.Sectors(hv, I.Cut("updn"), 3, 3, host_only=True)) == E.ECUT_EUNSUPPORTED
    h18 = I.hubbard_chain(18)
    assert _status(lambda: E.Sectors(h18, I.Cut("spatial", 1), 2, 2, host_only=True)) == E.ECUT_EUNSUPPORTED
    assert _status(lambda: E.Sectors(h, I.Cut("updn"), 3, 7, host_only=True)) == E.ECUT_EINVAL
    bad = I.Model("spin", 4, np.array([[0, 0]], dtype=np.int32), jxy=np.ones(1), jz=np.ones(1))
    assert _status(lambda: E.Sectors(bad, I.Cut("spatial", 0b11), 2, host_only=True)) == E.ECUT_EINVAL
    big = I.xxz_chain(40)
    assert _status(lambda: E.Sectors(big, I.Cut("spatial", (1 << 35) - 1), 20, host_only=True)) == E.ECUT_EUNSUPPORTED
    # device calls on a host-only handle are rejected before any device work
    S = E.Sectors(m, I.Cut("spatial", 0b111), 3, host_only=True)
    st = E.lib().ecut_apply_H(S.h, None, None, None)
    assert st == E.ECUT_EINVAL


def test_bench_names_every_kernel_variant():
    # the benchmark names the kernel of every tuning the autotuner may choose
    import bench
    S3 = E.Sectors.from_problem(I.hubbard16(), host_only=True)
    names = set()
    assert S3.info.kernel_flags & 16
    for v in range(6):
        S3.set_tuning(0, 1, 0, v)
        names.add(bench.kernel_name(S3))
    assert names == {"k_hub3", "k_hub", "k_hub2", "k_upslab+k_hub3", "k_hubrow", "k_hubseg"}
    S4 = E.Sectors.from_problem(I.j1j2_6x5(), host_only=True)
    for v, want in ((0, "k_spin"), (1, "k_rows"), (2, "k_spinL+k_spinR")):
        S4.set_tuning(0, 0, 0, v)
        assert bench.kernel_name(S4) == want


def test_bench_traffic_lookup(tmp_path, monkeypatch):
    """The benchmark takes HBM traffic from a counter summary only when the
    summary was made from the current kernel source, and reports the launch
    tuning of its counter runs beside it."""
    import json
    import bench
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    assert bench.traffic_from_profile("k_x", "w", 0) == (None, None)
    d = {"kernel_hash": h, "bytes_per_launch": 123.0,
         "commands": {"fetch": "rocprofv3 --pmc FETCH_SIZE -o run -- python3 bench.py --tuning 0,8,8,0 --steps 3"}}
    path = tmp_path / "profiles" / "k_x_w_traffic.json"
    path.write_text(json.dumps(d))
    assert bench.traffic_from_profile("k_x", "w", 0) == (123.0, "0,8,8,0")
    d["commands"]["fetch"] = "rocprofv3 --pmc FETCH_SIZE -o run -- python3 bench.py"
    path.write_text(json.dumps(d))
    assert bench.traffic_from_profile("k_x", "w", 0) == (123.0, None)
    d["kernel_hash"] = "0" * 16
    path.write_text(json.dumps(d))
    assert bench.traffic_from_profile("k_x", "w", 0) == (None, None)


def test_kernel_hash_follows_code_not_comments(tmp_path, monkeypatch):
    """The hash that guards the counter summaries changes with the kernels'
    code and not with their comments or spacing."""
    import shutil
    import bench
    src = os.path.join(ROOT, "paper_2605_07621_amd", "csrc")
    dst = tmp_path / "paper_2605_07621_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("kernels.hip", "kernels.h", "ecut_internal.h", "sectors.cpp"):
        shutil.copy(os.path.join(src, name), dst / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    k = dst / "kernels.h"
    text = k.read_text()
    k.write_text(text.replace("namespace ecut {", "namespace ecut {  // a comment\n/* and a\n block */\n", 1))
    assert bench.kernel_source_hash() == h0
    k.write_text(text.replace("constexpr int HUBD_NB = 8;", "constexpr int HUBD_NB = 16;", 1))
    assert "HUBD_NB = 16" in k.read_text()
    assert bench.kernel_source_hash() != h0


def test_option_structs_match_header():
    # the binding's ctypes structs follow the header's field order and types
    import ctypes
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "ecut.h")).read()
    ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double,
             "uint64_t": ctypes.c_uint64}
    for cname, py in (("ecut_lanczos_opts", E.LanczosOpts), ("ecut_server_opts", E.ServerOpts),
                      ("ecut_tuning", E.Tuning), ("ecut_lanczos_stats", E.LanczosStats), ("ecut_result", E.Result)):
        body = re.search(r"typedef struct " + cname + r" \{(.*?)\} " + cname + ";", hdr, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"(int32_t|int64_t|double|uint64_t)\s+(\w+);", body)
        assert [f for f, _ in py._fields_] == [n for _, n in fields], cname
        assert [t for _, t in py._fields_] == [ctype[ty] for ty, _ in fields], cname


def test_spin_tile_tuning_host():
    # the short-row tile of the spin kernel is a tuning field: validated, kept
    # on the handle, and it leaves the Lanczos workspace size unchanged
    S = E.Sectors.from_problem(I.j1j2_6x5(), host_only=True)
    assert S.info.kernel_flags & 4
    ws = S.lanczos_workspace(40)
    for tile in (1, 64, 128, 256, 512, 0):
        S.set_tuning(0, 0, 0, 0, tile)
        assert S.get_tuning()["tile"] == tile
        assert S.lanczos_workspace(40) == ws
    for bad in (-1, 513, 4096):
        assert _status(lambda: S.set_tuning(0, 0, 0, 0, bad)) == E.ECUT_EINVAL
    S.set_tuning(0, 0, 1, 0, 128)                # segments dealt to the XCDs
    assert S.get_tuning()["row_order"] == 1 and S.lanczos_workspace(40) == ws
    assert _status(lambda: S.set_tuning(0, 0, 2, 0, 0)) == E.ECUT_EINVAL
    S.set_tuning(0, 0, 0, 0, 0)
    assert S.get_tuning()["tile"] == 0          # a rejected tuning changes nothing
    # problems that do not run the spin kernel take no tile
    H = E.Sectors.from_problem(I.hubbard12(), host_only=True)
    assert _status(lambda: H.set_tuning(0, 1, 0, 0, 128)) == E.ECUT_EUNSUPPORTED
    G = E.Sectors.from_problem(I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", 0b111), 10), host_only=True)
    assert not G.info.kernel_flags & 4
    assert _status(lambda: G.set_tuning(0, 0, 0, 0, 64)) == E.ECUT_EUNSUPPORTED


def test_whole_row_group_size_tuning_host():
    """Hubbard variant 4 takes its work-group size in the tile field: 256,
    512 or 1024 threads, as long as a row fits 14 columns per thread."""
    H = E.Sectors.from_problem(I.hubbard12(), host_only=True)      # rows of 924 columns
    assert H.info.kernel_flags & 8
    for tile in (256, 512, 1024, 0):
        H.set_tuning(0, 8, 0, 4, tile)
        assert H.get_tuning()["tile"] == tile and H.get_tuning()["variant"] == 4
    for bad in (-1, 128, 300, 2048):
        assert _status(lambda: H.set_tuning(0, 8, 0, 4, bad)) == E.ECUT_EINVAL
    assert _status(lambda: H.set_tuning(0, 8, 0, 0, 256)) == E.ECUT_EUNSUPPORTED   # other variants: tile 0
    C3 = E.Sectors.from_problem(I.hubbard16(), host_only=True)      # rows of 12,870 columns
    assert C3.info.kernel_flags & 8
    for tile in (256, 512):
        assert _status(lambda: C3.set_tuning(0, 8, 0, 4, tile)) == E.ECUT_EUNSUPPORTED
    C3.set_tuning(0, 8, 0, 4, 1024)
    assert C3.get_tuning()["tile"] == 1024


def _spatial_hubbard_cases():
    rng = np.random.default_rng(2605)
    out = []
    for n, nu, nd in ((2, 1, 1), (4, 2, 1), (5, 2, 3), (6, 3, 3), (7, 4, 2), (8, 3, 5), (9, 4, 4), (10, 5, 5)):
        m = I.random_extended_hubbard_model(rng, n)
        mask = int(rng.integers(1, (1 << n) - 1))
        out.append((m, mask, nu, nd))
    # whole system on one side, empty sectors on the other, the chain's half cut
    out.append((I.hubbard_chain(6, V=1.0), (1 << 6) - 1, 3, 2))
    out.append((I.hubbard_chain(6, V=1.0), 0, 2, 3))
    out.append((I.hubbard_chain(10, V=1.0), I.left_mask_first(5), 5, 5))
    out.append((I.hubbard_chain(8, V=1.0), 0b10101010, 0, 4))
    return out


@pytest.mark.parametrize("case", _spatial_hubbard_cases(), ids=lambda c: f"{c[0].name}-{c[1]:#x}-{c[2]}-{c[3]}")
def test_spatial_hubbard_layout_and_signs_bit_exact(case):
    """Blocks (N_up_L, N_dn_L), positions and fermion signs of the spatial
    Hubbard cut against the oracle's signed map (itself pinned against
    fermionic Kronecker products of the two parts)."""
    m, mask, nu, nd = case
    S = E.Sectors(m, I.Cut("spatial", mask), nu, nd, host_only=True)
    pos, sign, ob = O.Sector(m, nu, nd).bipartite_signed(mask)
    blocks, lab = S.blocks(), S.labels()
    assert S.dim == len(pos)
    assert blocks.shape[0] == ob.shape[0]
    np.testing.assert_array_equal(lab[:, 0], ob[:, 0])
    np.testing.assert_array_equal(lab[:, 1], ob[:, 1])
    np.testing.assert_array_equal(lab[:, 2], nu - ob[:, 0])
    np.testing.assert_array_equal(lab[:, 3], nd - ob[:, 1])
    np.testing.assert_array_equal(blocks[:, 2], ob[:, 2])
    np.testing.assert_array_equal(blocks[:, 3], ob[:, 3])
    np.testing.assert_array_equal(blocks[:, 4], ob[:, 4])
    np.testing.assert_array_equal(S.canonical_positions(), pos)
    np.testing.assert_array_equal(S.canonical_signs(), sign)


def test_canonical_signs_are_one_without_fermion_reordering():
    for p in (I.Problem(I.xxz_chain(8), I.Cut("spatial", 0b1111), 4), I.hubbard12()):
        S = E.Sectors.from_problem(p, host_only=True)
        assert np.all(S.canonical_signs() == 1)


def test_tuning_validation_host():
    """Tunings outside what a handle's kernels take are refused before any
    device work: two-pass rows per item, the slabs side by side of variant 7,
    variant 2 on problems without two-pass tables."""
    C3 = E.Sectors.from_problem(I.hubbard16(), host_only=True)
    for t in ((8, 8, 8, 7, 0), (8, 8, 8, 7, 2), (8, 8, 8, 7, 4), (32, 8, 8, 7, 0), (0, 8, 1, 6, 16)):
        C3.set_tuning(*t)
    for t in ((33, 8, 8, 7, 0), (16, 8, 8, 7, 4), (8, 8, 8, 7, 3), (8, 8, 1, 6, 3)):
        assert _status(lambda: C3.set_tuning(*t)) == E.ECUT_EINVAL, t
    C4 = E.Sectors.from_problem(I.j1j2_6x5(), host_only=True)
    C4.set_tuning(32, 8, 0, 2, 0)
    assert _status(lambda: C4.set_tuning(33, 8, 0, 2, 0)) == E.ECUT_EINVAL
    assert _status(lambda: C4.set_tuning(0, 8, 0, 3, 0)) == E.ECUT_EINVAL
    H = E.Sectors.from_problem(I.hubbard14_spatial(), host_only=True)
    H.set_tuning(8, 8, 0, 2, 0)
    H.set_tuning(0, 0, 0, 0, 0)
    assert _status(lambda: H.set_tuning(0, 0, 0, 2, 64)) != E.ECUT_OK   # every row is its own item
    wide = E.Sectors.from_problem(I.Problem(I.xxz_chain(20, 1.0, 1.0), I.Cut("spatial", 0b111), 10), host_only=True)
    assert not wide.info.kernel_flags & 64
    assert _status(lambda: wide.set_tuning(0, 0, 0, 2, 0)) != E.ECUT_OK


def test_server_two_lane_option_checks():
    # a two-lane server (large_dim > 0) does not replay graphs, and a negative
    # threshold is refused; both are checked before any device call
    for kw in (dict(use_graph=True, large_dim=100), dict(large_dim=-1)):
        with pytest.raises(E.EcutError) as ei:
            E.Server(1 << 20, **kw)
        assert ei.value.status == E.ECUT_EINVAL, kw
