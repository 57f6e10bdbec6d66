"""Pins of the CPU oracle against things other than itself.

Each test ties an oracle function to mathematics the paper fixes or to an
independent construction:
  - basis enumeration vs brute force over all 2^n words and vs binomials;
  - Hamiltonian entries vs dense Kronecker-product constructions (Pauli
    matrices for spins; Jordan-Wigner strings for fermions), which share no
    code with the oracle's term-by-term sign counting;
  - the bipartite map vs the block identity of Eq. (2) with the
    Vec-Kronecker rule (left operator from the left, right operator from
    the right) built from independently enumerated subsystem sectors;
  - Lanczos energies vs closed forms (free fermions, XX chain, two-site
    problems) and vs dense diagonalisation;
  - Sturm bisection vs a library tridiagonal eigensolver.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2605_07621_amd import inputs as I


# ---------------------------------------------------------------- bases

@pytest.mark.parametrize("n", [1, 2, 5, 8, 12, 16])
def test_enumeration_matches_bruteforce(n):
    for k in range(n + 1):
        w = O.enumerate_basis("spin", n, k)
        assert len(w) == math.comb(n, k)
        np.testing.assert_array_equal(w, O.enumerate_bruteforce(n, k))


def test_hubbard_enumeration_is_up_major_product():
    L = 6
    w = O.enumerate_basis("hubbard", L, 2, 3)
    assert len(w) == math.comb(6, 2) * math.comb(6, 3)
    assert np.all(np.diff(w.astype(np.int64)) > 0)
    up = O.enumerate_bruteforce(L, 2)
    dn = O.enumerate_bruteforce(L, 3)
    ref = np.array([(int(a) << L) | int(b) for a in up for b in dn], dtype=np.uint64)
    np.testing.assert_array_equal(w, ref)


def test_sector_sizes_of_measured_workloads():
    # 16-site chain at Sz=0: C(16,8); 12-site Hubbard half filling: C(12,6)^2;
    # 16-site Hubbard: C(16,8)^2; 6x5 lattice at Sz=0: C(30,15).
    assert O.sector_size("spin", 16, 8) == 12870
    assert O.sector_size("hubbard", 12, 6, 6) == 924 * 924 == 853776
    assert O.sector_size("hubbard", 16, 8, 8) == 12870 ** 2 == 165636900
    assert O.sector_size("spin", 30, 15) == 155117520


def test_find():
    w = O.enumerate_basis("spin", 10, 4)
    s = O.Sector(I.heisenberg_chain(10), 4)
    for i in [0, 1, 57, len(w) - 1]:
        assert s.find(w[i]) == i
    assert s.find(0b1111000000) == list(w).index(0b1111000000)
    assert s.find(0b111) == -1


# ---------------------------------------------------------------- spin H vs Pauli Kronecker products

SZ = np.diag([-0.5, 0.5])          # local basis: index 0 = down, 1 = up (bit set)
SP = np.array([[0.0, 0.0], [1.0, 0.0]])   # S+ |down> = |up>
SM = SP.T
ID2 = np.eye(2)


def site_op(op, i, n):
    """Operator on site i of n; matrix index = sum_i bit_i 2^i."""
    out = np.array([[1.0]])
    for s in range(n - 1, -1, -1):
        out = np.kron(out, op if s == i else ID2)
    return out


def dense_spin(model):
    n = model.n_sites
    H = np.zeros((2 ** n, 2 ** n))
    for (i, j), jxy, jz in zip(model.bonds, model.jxy, model.jz):
        H += jz * site_op(SZ, i, n) @ site_op(SZ, j, n)
        H += 0.5 * jxy * (site_op(SP, i, n) @ site_op(SM, j, n) + site_op(SM, i, n) @ site_op(SP, j, n))
    return H


@pytest.mark.parametrize("seed,n", [(1, 4), (2, 6), (3, 7), (4, 8)])
def test_spin_hamiltonian_vs_pauli_kron(seed, n):
    rng = np.random.default_rng(seed)
    m = I.random_spin_model(rng, n)
    Hfull = dense_spin(m)
    for k in range(n + 1):
        s = O.Sector(m, k)
        idx = s.words.astype(np.int64)
        np.testing.assert_allclose(s.dense(), Hfull[np.ix_(idx, idx)], atol=1e-14, rtol=0)


def test_spin_sector_blocks_cover_full_matrix():
    # Sz conservation: the Kronecker H has no element between sectors.
    m = I.random_spin_model(np.random.default_rng(9), 6)
    Hfull = dense_spin(m)
    w = np.arange(2 ** 6)
    pc = np.array([bin(x).count("1") for x in w])
    assert np.abs(Hfull[pc[:, None] != pc[None, :]]).max() == 0.0


# ---------------------------------------------------------------- Hubbard H vs Jordan-Wigner strings

ZF = np.diag([1.0, -1.0])          # (-1)^n
AF = np.array([[0.0, 1.0], [0.0, 0.0]])   # a|1> = |0>


def jw_annihilator(m, M):
    """c_m = Z_0 ... Z_{m-1} a_m on M modes; matrix index = sum_m n_m 2^m."""
    out = np.array([[1.0]])
    for k in range(M - 1, -1, -1):
        op = AF if k == m else (ZF if k < m else ID2)
        out = np.kron(out, op)
    return out


def dense_hubbard_word_basis(model):
    """Dense Hubbard H via Jordan-Wigner, modes ordered (0,up)..(L-1,up),
    (0,dn)..(L-1,dn), re-indexed to the word (up << L) | dn."""
    L = model.n_sites
    M = 2 * L
    c = [jw_annihilator(m, M) for m in range(M)]
    H = np.zeros((2 ** M, 2 ** M))
    for (i, j), t in zip(model.bonds, model.t):
        for sp in range(2):
            a, b = sp * L + i, sp * L + j
            H += -t * (c[a].T @ c[b] + c[b].T @ c[a])
    for s in range(L):
        H += model.u[s] * (c[s].T @ c[s]) @ (c[L + s].T @ c[L + s])
    # mode-bit index -> word index: up site s (mode s) is word bit L+s, dn site s (mode L+s) is bit s
    perm = np.zeros(2 ** M, dtype=np.int64)
    for idx in range(2 ** M):
        word = 0
        for m in range(M):
            if (idx >> m) & 1:
                word |= 1 << ((L + m) if m < L else (m - L))
        perm[idx] = word
    Hw = np.zeros_like(H)
    Hw[np.ix_(perm, perm)] = H
    return Hw


@pytest.mark.parametrize("seed,L", [(11, 2), (12, 3), (13, 4), (14, 4)])
def test_hubbard_hamiltonian_vs_jordan_wigner(seed, L):
    rng = np.random.default_rng(seed)
    m = I.random_hubbard_model(rng, L, n_bonds=min(L * (L - 1) // 2, 2 * L))
    Hfull = dense_hubbard_word_basis(m)
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = O.Sector(m, nu, nd)
            idx = s.words.astype(np.int64)
            np.testing.assert_allclose(s.dense(), Hfull[np.ix_(idx, idx)], atol=1e-14, rtol=0)


def test_long_range_hop_carries_fermion_sign():
    # A hop 0<->2 over an occupied site 1 must pick up a minus sign relative
    # to the same hop over an empty site (same-spin electrons only).
    m = I.Model("hubbard", 3, np.array([[0, 2]], dtype=np.int32), t=np.array([1.0]), u=np.zeros(3))
    s = O.Sector(m, 2, 0)
    H = s.dense()
    L = 3
    w_a = (0b011 << L)   # up on sites 0,1
    w_b = (0b110 << L)   # up on sites 1,2
    ia, ib = s.find(w_a), s.find(w_b)
    assert H[ia, ib] == pytest.approx(+1.0)   # -t * (-1)
    s0 = O.Sector(m, 1, 0)
    H0 = s0.dense()
    assert H0[s0.find(0b001 << L), s0.find(0b100 << L)] == pytest.approx(-1.0)


@pytest.mark.parametrize("kind", ["spin", "hubbard"])
def test_hermiticity(kind):
    rng = np.random.default_rng(5)
    if kind == "spin":
        s = O.Sector(I.random_spin_model(rng, 10), 5)
    else:
        s = O.Sector(I.random_hubbard_model(rng, 5), 2, 3)
    phi = rng.standard_normal(s.n)
    psi = rng.standard_normal(s.n)
    lhs = phi @ s.apply(psi)
    rhs = s.apply(phi) @ psi
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_row_generator_matches_csr():
    rng = np.random.default_rng(6)
    s = O.Sector(I.random_hubbard_model(rng, 6), 3, 2)
    x = rng.standard_normal(s.n)
    y1 = s.apply(x, use_csr=True)
    y2 = s.apply(x, use_csr=False)
    np.testing.assert_array_equal(y1, y2)
    rows = rng.integers(0, s.n, 50)
    np.testing.assert_array_equal(s.apply_rows(x, rows), y1[rows])


# ---------------------------------------------------------------- bipartite map vs Eq. (2) block identity

def _submodel_spin(model, sites):
    """Restrict a spin model to the bonds inside `sites`, renumbered 0..k-1."""
    idx = {s: k for k, s in enumerate(sites)}
    keep = [b for b in range(len(model.bonds)) if model.bonds[b][0] in idx and model.bonds[b][1] in idx]
    bonds = np.array([[idx[model.bonds[b][0]], idx[model.bonds[b][1]]] for b in keep], dtype=np.int32).reshape(-1, 2)
    return I.Model("spin", len(sites), bonds, jxy=model.jxy[keep], jz=model.jz[keep])


@pytest.mark.parametrize("seed,n,left", [(21, 8, [0, 1, 2]), (22, 9, [1, 4, 5, 8]), (23, 10, [0, 2, 4, 6, 8])])
def test_spatial_bipartite_map_vs_block_identity(seed, n, left):
    """With no bond across the cut, H = H_L x 1 + 1 x H_R, so in the
    bipartite layout every block obeys Y_q = H_L^{q_l} Psi_q + Psi_q H_R^{q_r T}
    (the Vec-Kronecker rule for column-stacked blocks)."""
    rng = np.random.default_rng(seed)
    right = [s for s in range(n) if s not in left]
    full = I.random_spin_model(rng, n, n_bonds=3 * n)
    keep = [b for b in range(len(full.bonds))
            if (full.bonds[b][0] in left) == (full.bonds[b][1] in left)]
    model = I.Model("spin", n, full.bonds[keep], jxy=full.jxy[keep], jz=full.jz[keep])
    mask = sum(1 << s for s in left)
    for n_up in range(n + 1):
        s = O.Sector(model, n_up)
        pos, blocks = s.bipartite("spatial", mask)
        assert sorted(pos.tolist()) == list(range(s.n))
        x = rng.standard_normal(s.n)
        y = s.apply(x)
        xb = np.empty(s.n); xb[pos] = x
        yb = np.empty(s.n); yb[pos] = y
        mL, mR = _submodel_spin(model, left), _submodel_spin(model, right)
        for q_l, dL, dR, off in blocks:
            HL = O.Sector(mL, int(q_l)).dense()
            HR = O.Sector(mR, n_up - int(q_l)).dense()
            P = xb[off:off + dL * dR].reshape(dL, dR)
            np.testing.assert_allclose(yb[off:off + dL * dR].reshape(dL, dR), HL @ P + P @ HR.T,
                                       atol=1e-12, rtol=0)


def test_spatial_cut_cross_term_vs_kron():
    """One bond across the cut: Y = [H_L x 1 + 1 x H_R + sum_m L_m x R_m] Psi
    evaluated with np.kron on each block pair (q, k) must agree with the
    oracle's full H in bipartite order."""
    rng = np.random.default_rng(31)
    n, left = 6, [0, 1, 2]
    bonds = np.array([[0, 1], [1, 2], [3, 4], [4, 5], [2, 3]], dtype=np.int32)
    model = I.Model("spin", n, bonds, jxy=rng.uniform(0.5, 1.5, 5), jz=rng.uniform(0.5, 1.5, 5))
    n_up = 3
    s = O.Sector(model, n_up)
    pos, blocks = s.bipartite("spatial", 0b000111)
    Hb = np.zeros((s.n, s.n))
    Hb[np.ix_(pos, pos)] = s.dense()
    # Independent construction: full 2^6 Kronecker H, then pick rows/cols by
    # the (l, r) words of each block, L word = bits of sites 0..2, R word = sites 3..5.
    Hk = dense_spin(model)
    order = []
    for q_l, dL, dR, off in blocks:
        lw = O.enumerate_bruteforce(3, int(q_l))
        rw = O.enumerate_bruteforce(3, n_up - int(q_l))
        for a in lw:
            for b in rw:
                order.append(int(a) | (int(b) << 3))
    order = np.array(order)
    np.testing.assert_allclose(Hb, Hk[np.ix_(order, order)], atol=1e-14, rtol=0)


def test_updn_bipartite_map_vs_block_identity():
    """Up/down cut at U=0: H = H_up x 1 + 1 x H_dn, so Y = H_up Psi + Psi H_dn^T
    with Psi[up, dn]; at U != 0 the extra term is diagonal in (up, dn)."""
    rng = np.random.default_rng(41)
    L = 6
    m = I.random_hubbard_model(rng, L, n_bonds=8)
    m0 = I.Model("hubbard", L, m.bonds, t=m.t, u=np.zeros(L))
    nu, nd = 3, 2
    s = O.Sector(m0, nu, nd)
    pos, blocks = s.bipartite("updn")
    np.testing.assert_array_equal(pos, np.arange(s.n))
    assert blocks.tolist() == [[nu, math.comb(L, nu), math.comb(L, nd), 0]]
    Hup = O.Sector(m0, nu, 0).dense()
    Hdn = O.Sector(m0, 0, nd).dense()
    x = rng.standard_normal(s.n)
    P = x.reshape(math.comb(L, nu), math.comb(L, nd))
    np.testing.assert_allclose(s.apply(x).reshape(P.shape), Hup @ P + P @ Hdn.T, atol=1e-12, rtol=0)
    # the U part is diagonal: H(U) - H(0) has no off-diagonal element
    D = O.Sector(m, nu, nd).dense() - s.dense()
    assert np.abs(D - np.diag(np.diag(D))).max() == 0.0


# ---------------------------------------------------------------- energies: closed forms and dense

def free_fermion_chain_energy(L, n_per_spin, t=1.0, spins=2):
    eps = np.sort(-2.0 * t * np.cos(np.arange(1, L + 1) * np.pi / (L + 1)))
    return spins * eps[:n_per_spin].sum()


def test_u0_hubbard_12_sites_closed_form():
    p = I.hubbard12()
    m = I.hubbard_chain(12, 1.0, 0.0)
    s = O.Sector(m, 6, 6)
    e, a, b = s.lanczos(I.psi(p.meta["seed"] + 1, s.n), 200)
    ref = free_fermion_chain_energy(12, 6)
    assert ref == pytest.approx(-14.592459621117511, abs=1e-12)
    assert abs(e[-1] - ref) <= 1e-10


def test_xx_chain_closed_form():
    n = 16
    m = I.xxz_chain(n, 1.0, 0.0)
    s = O.Sector(m, n // 2)
    e, _, _ = s.lanczos(I.psi(7, s.n), 150)
    # Jordan-Wigner: free fermions with hopping J/2, levels J cos(k pi/(N+1)).
    lev = np.sort(np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert abs(e[-1] - lev[: n // 2].sum()) <= 1e-10


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 8.0])
def test_two_site_hubbard_closed_form(U):
    m = I.hubbard_chain(2, 1.0, U)
    s = O.Sector(m, 1, 1)
    ev = np.linalg.eigvalsh(s.dense())
    assert ev[0] == pytest.approx((U - math.sqrt(U * U + 16.0)) / 2.0, abs=1e-13)


def test_two_site_heisenberg_singlet():
    s = O.Sector(I.heisenberg_chain(2), 1)
    assert np.linalg.eigvalsh(s.dense())[0] == pytest.approx(-0.75, abs=1e-15)


@pytest.mark.parametrize("kind,seed", [("spin", 1), ("spin", 2), ("hubbard", 3), ("hubbard", 4)])
def test_lanczos_vs_dense(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "spin":
        s = O.Sector(I.random_spin_model(rng, 10), 5)
    else:
        s = O.Sector(I.random_hubbard_model(rng, 5), 2, 3)
    ev = np.linalg.eigvalsh(s.dense())
    e, a, b = s.lanczos(rng.standard_normal(s.n), min(s.n, 120), reorth=True)
    assert abs(e[-1] - ev[0]) <= 1e-10
    # Cauchy interlacing: the lowest Ritz value never increases
    assert np.all(np.diff(e) <= 1e-12)


def test_heisenberg16_dense_vs_lanczos():
    p = I.heisenberg16()
    s = O.Sector(p.model, 8)
    e, _, _ = s.lanczos(I.psi(p.meta["seed"] + 1, s.n), 100)
    rp, col, val = s.csr()
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    H = sp.csr_matrix((val, col, rp), shape=(s.n, s.n))
    ref = sla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(e[-1] - ref) <= 1e-10


@pytest.mark.parametrize("m", [1, 2, 7, 40])
def test_bisection_vs_eigvalsh(m):
    rng = np.random.default_rng(m)
    a = rng.standard_normal(m)
    b = rng.standard_normal(max(m - 1, 0))
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    ev = np.linalg.eigvalsh(T)
    for k in range(m):
        assert O.tridiag_eig(a, b, k) == pytest.approx(ev[k], abs=1e-13)


@pytest.mark.parametrize("tol", [1e-9, 1e-12, 1e-14])
def test_lanczos_stopping_rule(tol):
    """The oracle's Lanczos stops once the lowest Ritz value has moved by at
    most tol over three steps in a row, and not before: the energies it
    returns are those of a fixed-step run (same arithmetic) up to that step,
    the last three moves are within tol, no earlier three-step run is, and
    the energy agrees with dense diagonalisation (eigh) within 1e-12 for the
    tight tolerances, as a run continued well past convergence does."""
    p = I.Problem(I.xxz_chain(12, 1.0, 0.8), I.Cut("spatial", I.left_mask_first(6)), 6)
    s = O.Sector(p.model, p.n_up)
    v0 = I.psi(31, s.n)
    e_fixed, _, _ = s.lanczos(v0, 300)
    e_tol, _, _ = s.lanczos(v0, 300, tol=tol)
    k = len(e_tol)
    assert 4 <= k < 300
    np.testing.assert_array_equal(e_tol, e_fixed[:k])
    moves = np.abs(np.diff(e_tol))
    assert np.all(moves[-3:] <= tol)
    run = 0
    for m in moves[:-1]:
        run = run + 1 if m <= tol else 0
        assert run < 3
    w0 = np.linalg.eigvalsh(s.dense())[0]
    assert abs(e_fixed[-1] - w0) <= 1e-12
    if tol <= 1e-12:
        assert abs(e_tol[-1] - w0) <= 1e-12


def test_csr_rows_block_matches_full_csr():
    """A CSR block of a row range (the host baseline's sample) is the same
    rows of the full CSR, and its product gives the same entries of H x."""
    p = I.hubbard_chain(8, 1.0, 3.0)
    s = O.Sector(p, 4, 3)
    rp, col, val = s.csr()
    r0, r1 = 17, 901
    rb, cb, vb = s.csr_rows(r0, r1)
    np.testing.assert_array_equal(rb, rp[r0:r1 + 1] - rp[r0])
    np.testing.assert_array_equal(cb, col[rp[r0]:rp[r1]])
    np.testing.assert_array_equal(vb, val[rp[r0]:rp[r1]])
    x = I.psi(5, s.n)
    np.testing.assert_array_equal(O.spmv_csr(rb, cb, vb, x), s.apply(x)[r0:r1])


# ---------------------------------------------------------------- entanglement spectrum

def _full_matrix(words, psi, n_sites, left_mask):
    """psi as the full 2^n_L x 2^n_R matrix M[l, r] (no symmetry blocks),
    by direct bit selection: the reference for the block-resolved
    spectrum."""
    lsites = [i for i in range(n_sites) if (left_mask >> i) & 1]
    rsites = [i for i in range(n_sites) if not (left_mask >> i) & 1]
    M = np.zeros((1 << len(lsites), 1 << len(rsites)))
    for w, a in zip(words, psi):
        w = int(w)
        l = sum(((w >> s) & 1) << k for k, s in enumerate(lsites))
        r = sum(((w >> s) & 1) << k for k, s in enumerate(rsites))
        M[l, r] = a
    return M


@pytest.mark.parametrize("mask", [0b0000011111, 0b1010010110, 0b1])
def test_entanglement_blocks_vs_full_matrix_svd(mask):
    """The union of the block spectra equals the squared singular values of
    the whole state matrix over the cut (normalised), for random states."""
    p = I.xxz_chain(10, 1.0, 0.7)
    s = O.Sector(p, 5)
    psi = I.psi(41, s.n)
    e = O.entanglement(s, psi, "spatial", mask)
    sv = np.linalg.svd(_full_matrix(s.words, psi, 10, mask), compute_uv=False)
    ref = np.sort(sv * sv / (psi @ psi))[::-1]
    got = np.sort(np.concatenate(e["lam"]))[::-1]
    k = min(len(ref), len(got))
    np.testing.assert_allclose(got[:k], ref[:k], atol=1e-14)
    assert np.all(ref[k:] < 1e-14) and np.all(got[k:] < 1e-14)
    assert abs(e["w_q"].sum() - 1.0) < 1e-13


def test_entanglement_product_state_and_singlet():
    """A basis state has one Schmidt value 1 (xi = 0, zero entropy); the
    two-site singlet has two equal weights 1/2 in two sectors (entropy log 2,
    W_q = 1/2 each, weight IPR 2)."""
    p = I.xxz_chain(8, 1.0, 1.0)
    s = O.Sector(p, 4)
    psi = np.zeros(s.n)
    psi[17] = 3.0
    e = O.entanglement(s, psi, "spatial", 0b00001111)
    lam = np.concatenate(e["lam"])
    assert np.sum(lam > 1e-15) == 1 and abs(lam.max() - 1.0) < 1e-15 and abs(e["entropy"]) < 1e-15
    two = I.heisenberg_chain(2)
    s2 = O.Sector(two, 1)
    w, V = np.linalg.eigh(s2.dense())
    assert abs(w[0] + 0.75) < 1e-14
    e2 = O.entanglement(s2, V[:, 0], "spatial", 0b01, parts=np.array([0, 1]))
    np.testing.assert_allclose([l[0] for l in e2["lam"]], [0.5, 0.5], atol=1e-15)
    np.testing.assert_allclose(e2["w_q"], [0.5, 0.5], atol=1e-15)
    assert abs(e2["entropy"] - np.log(2)) < 1e-14 and abs(e2["weight_ipr"] - 2.0) < 1e-13
    np.testing.assert_allclose(e2["w_p"], [0.25, 0.25], atol=1e-15)


def test_entanglement_hubbard_product_of_spin_words():
    """Up/down cut: a state that is a product of an up-spin and a down-spin
    amplitude vector has rank one; a sum of two such products with
    orthogonal factors has the two weights of the sum."""
    p = I.hubbard_chain(6, 1.0, 2.0)
    s = O.Sector(p, 3, 2)
    rng = np.random.default_rng(3)
    nu, nd = 20, 15
    a1, a2 = np.linalg.qr(rng.standard_normal((nu, 2)))[0].T
    b1, b2 = np.linalg.qr(rng.standard_normal((nd, 2)))[0].T
    psi = (0.8 * np.outer(a1, b1) + 0.6 * np.outer(a2, b2)).ravel()   # canonical order is up-major
    e = O.entanglement(s, psi, "updn")
    lam = e["lam"][0]
    np.testing.assert_allclose(lam[:2], [0.64, 0.36], atol=1e-14)
    assert np.all(lam[2:] < 1e-14)


def test_ground_state_vs_dense():
    p = I.xxz_chain(10, 1.0, 0.6)
    s = O.Sector(p, 5)
    e, g = O.ground_state(s, I.psi(2, s.n))
    w, V = np.linalg.eigh(s.dense())
    assert abs(e - w[0]) < 1e-12 and abs(abs(g @ V[:, 0]) - 1.0) < 1e-10


# ---------------------------------------------------------------- c+ / c and the continued fraction

def _dense_cdag_word_basis(L, site, spin):
    """c+_{site,spin} as a dense Jordan-Wigner matrix re-indexed to words."""
    M = 2 * L
    cd = jw_annihilator(spin * L + site, M).T
    perm = np.zeros(2 ** M, dtype=np.int64)
    for idx in range(2 ** M):
        word = 0
        for m in range(M):
            if (idx >> m) & 1:
                word |= 1 << ((L + m) if m < L else (m - L))
        perm[idx] = word
    out = np.zeros_like(cd)
    out[np.ix_(perm, perm)] = cd
    return out


@pytest.mark.parametrize("site,spin", [(0, 0), (2, 0), (3, 1), (1, 1)])
def test_apply_cdag_vs_jordan_wigner(site, spin):
    """c+ and c between sectors equal the Jordan-Wigner matrices restricted
    to the two sectors (signs included), and {c, c+} = 1 on a sector."""
    L = 4
    m = I.hubbard_chain(L, 1.0, 2.0)
    cd = _dense_cdag_word_basis(L, site, spin)
    nu, nd = 2, 1
    src = O.Sector(m, nu, nd)
    dst = O.Sector(m, nu + (spin == 0), nd + (spin == 1))
    x = I.psi(7, src.n)
    i_s, i_d = src.words.astype(np.int64), dst.words.astype(np.int64)
    np.testing.assert_allclose(O.apply_cdag(src, dst, site, spin, True, x), cd[np.ix_(i_d, i_s)] @ x, atol=1e-15)
    xd = I.psi(8, dst.n)
    np.testing.assert_allclose(O.apply_cdag(dst, src, site, spin, False, xd), cd.T[np.ix_(i_s, i_d)] @ xd, atol=1e-15)
    # c c+ + c+ c = 1 on the source sector
    lower = O.Sector(m, nu - (spin == 0), nd - (spin == 1))
    y = O.apply_cdag(dst, src, site, spin, False, O.apply_cdag(src, dst, site, spin, True, x)) + \
        O.apply_cdag(lower, src, site, spin, True, O.apply_cdag(src, lower, site, spin, False, x))
    np.testing.assert_allclose(y, x, atol=1e-14)


@pytest.mark.parametrize("dagger", [True, False])
def test_continued_fraction_vs_lehmann(dagger):
    """Green's function of a 4-site Hubbard chain from the oracle's Lanczos
    coefficients (the whole Krylov space) against the Lehmann sum over the
    exact eigenstates of the target sector:
      G+(w) = sum_n |<n|c+|0>|^2 / (w + i eta + E0 - E_n),
      G-(w) = sum_n |<n|c|0>|^2 / (w + i eta - E0 + E_n)."""
    L = 4
    m = I.hubbard_chain(L, 1.0, 3.0)
    s0 = O.Sector(m, 2, 2)
    w0, V0 = np.linalg.eigh(s0.dense())
    e0, g0 = w0[0], V0[:, 0]
    s1 = O.Sector(m, 3 if dagger else 1, 2)
    phi = O.apply_cdag(s0, s1, 1, 0, dagger, g0)
    weight = phi @ phi
    w1, V1 = np.linalg.eigh(s1.dense())
    amp = (V1.T @ phi) ** 2
    omega = np.linspace(-8, 8, 41)
    eta = 0.1
    if dagger:
        lehmann = np.sum(amp[None, :] / (omega[:, None] + 1j * eta + e0 - w1[None, :]), axis=1)
    else:
        lehmann = np.sum(amp[None, :] / (omega[:, None] + 1j * eta - e0 + w1[None, :]), axis=1)
    _, a, b = s1.lanczos(phi, s1.n, reorth=True)
    g = O.continued_fraction(a, b, weight, e0, dagger, omega, eta)
    np.testing.assert_allclose(g, lehmann, atol=1e-11)
    # sum rule: the spectral weight integrates to |c+ psi0|^2
    assert abs(weight - amp.sum()) < 1e-13


# ---------------------------------------------------------------- extended Hubbard (V) and the spatial cut

def dense_ext_hubbard_word_basis(model):
    """dense_hubbard_word_basis plus V_b n_i n_j (n = n_up + n_dn) on every bond."""
    L = model.n_sites
    H = dense_hubbard_word_basis(model)
    if model.v is None:
        return H
    d = np.zeros(2 ** (2 * L))
    for w in range(2 ** (2 * L)):
        for (i, j), v in zip(model.bonds, model.v):
            ni = ((w >> (L + i)) & 1) + ((w >> i) & 1)
            nj = ((w >> (L + j)) & 1) + ((w >> j) & 1)
            d[w] += v * ni * nj
    return H + np.diag(d)


@pytest.mark.parametrize("seed,L", [(21, 3), (22, 4)])
def test_extended_hubbard_vs_jordan_wigner(seed, L):
    m = I.random_extended_hubbard_model(np.random.default_rng(seed), L, n_bonds=min(L * (L - 1) // 2, 2 * L))
    Hfull = dense_ext_hubbard_word_basis(m)
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = O.Sector(m, nu, nd)
            idx = s.words.astype(np.int64)
            np.testing.assert_allclose(s.dense(), Hfull[np.ix_(idx, idx)], atol=1e-14, rtol=0)


def _subsystem_ops(n):
    """Annihilators of a subsystem of n sites: modes (up 0..n-1, dn 0..n-1),
    Jordan-Wigner in that order; basis index = up_bits | dn_bits << n."""
    return [jw_annihilator(m, 2 * n) for m in range(2 * n)]


def bipartite_hubbard_kron(model, left_mask):
    """The extended Hubbard H on the bipartite Fock space L (x) R built from
    subsystem operators: an L mode acts as c_L (x) 1, an R mode as
    P_L (x) c_R with P_L = (-1)^(N_L) (the R operators pass the L ones), the
    L modes ordered before the R modes.  Returns (H, lsites, rsites)."""
    S = model.n_sites
    ls = [i for i in range(S) if (left_mask >> i) & 1]
    rs = [i for i in range(S) if not (left_mask >> i) & 1]
    nL, nR = len(ls), len(rs)
    cL, cR = _subsystem_ops(nL), _subsystem_ops(nR)
    dL, dR = 2 ** (2 * nL), 2 ** (2 * nR)
    PL = np.diag([(-1.0) ** bin(k).count("1") for k in range(dL)])
    IL, IR = np.eye(dL), np.eye(dR)

    def c(site, spin):
        if site in ls:
            return np.kron(cL[spin * nL + ls.index(site)], IR)
        return np.kron(PL, cR[spin * nR + rs.index(site)])

    H = np.zeros((dL * dR, dL * dR))
    for b, (i, j) in enumerate(model.bonds):
        for sp in range(2):
            H += -model.t[b] * (c(i, sp).T @ c(j, sp) + c(j, sp).T @ c(i, sp))
        if model.v is not None:
            ni = c(i, 0).T @ c(i, 0) + c(i, 1).T @ c(i, 1)
            nj = c(j, 0).T @ c(j, 0) + c(j, 1).T @ c(j, 1)
            H += model.v[b] * ni @ nj
    for s in range(S):
        H += model.u[s] * (c(s, 0).T @ c(s, 0)) @ (c(s, 1).T @ c(s, 1))
    return H, ls, rs


@pytest.mark.parametrize("seed,L,mask", [(31, 4, 0b0101), (32, 5, 0b10110), (33, 4, 0b0011), (34, 5, 0b00001),
                                         (35, 4, 0b1111)])
def test_spatial_hubbard_map_vs_fermionic_kron(seed, L, mask):
    """The oracle's signed canonical -> bipartite map of the spatial Hubbard
    cut, applied to its full-basis H, gives the block Hamiltonian of Eq. (2)
    built from subsystem fermion operators (with the parity string of the
    left part on every right operator), every sector and block."""
    m = I.random_extended_hubbard_model(np.random.default_rng(seed), L, n_bonds=min(L * (L - 1) // 2, 2 * L))
    Hk, ls, rs = bipartite_hubbard_kron(m, mask)
    nL, nR = len(ls), len(rs)
    dR_full = 2 ** (2 * nR)
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = O.Sector(m, nu, nd)
            pos, sign, blocks = s.bipartite_signed(mask)
            # Kronecker index of every bipartite position, block by block
            kidx = np.empty(s.n, dtype=np.int64)
            for a, b, d_l, d_r, off in blocks:
                lw = [w for w in range(2 ** (2 * nL)) if bin(w >> nL).count("1") == a and bin(w & ((1 << nL) - 1)).count("1") == b]
                rw = [w for w in range(2 ** (2 * nR)) if bin(w >> nR).count("1") == nu - a and bin(w & ((1 << nR) - 1)).count("1") == nd - b]
                assert len(lw) == d_l and len(rw) == d_r
                # subsystem word (up << n) | dn  ->  Jordan-Wigner index up | dn << n
                jl = [(w >> nL) | ((w & ((1 << nL) - 1)) << nL) for w in lw]
                jr = [(w >> nR) | ((w & ((1 << nR) - 1)) << nR) for w in rw]
                for r_i, l in enumerate(jl):
                    kidx[off + r_i * d_r: off + (r_i + 1) * d_r] = np.asarray(jl[r_i]) * dR_full + np.asarray(jr)
            Hc = s.dense()
            Hb = np.zeros_like(Hc)
            Hb[np.ix_(pos, pos)] = Hc * np.outer(sign, sign)
            np.testing.assert_allclose(Hb, Hk[np.ix_(kidx, kidx)], atol=1e-13, rtol=0, err_msg=f"{nu},{nd}")


@pytest.mark.parametrize("seed,L,mask,nu,nd", [(41, 4, 0b0101, 2, 2), (42, 5, 0b10110, 2, 3), (43, 5, 0b00111, 3, 2)])
def test_spatial_hubbard_entanglement_vs_fermionic_kron(seed, L, mask, nu, nd):
    """Entanglement spectrum across the fermionic mode partition of a spatial
    Hubbard cut: the oracle's (its signed blocks of the ground state) equals
    the squared singular values of the ground state of the Kronecker-built H
    (subsystem fermion operators, no layout map) reshaped to L x R."""
    m = I.random_extended_hubbard_model(np.random.default_rng(seed), L, n_bonds=min(L * (L - 1) // 2, 2 * L))
    Hk, ls, rs = bipartite_hubbard_kron(m, mask)
    nL, nR = len(ls), len(rs)
    dL, dR = 2 ** (2 * nL), 2 ** (2 * nR)
    # number sector in the Kronecker basis: index = jl * dR + jr, each part
    # a Jordan-Wigner index up | dn << n
    def counts(j, n):
        return bin(j & ((1 << n) - 1)).count("1"), bin(j >> n).count("1")
    sel = [k for k in range(dL * dR)
           if counts(k // dR, nL)[0] + counts(k % dR, nR)[0] == nu and counts(k // dR, nL)[1] + counts(k % dR, nR)[1] == nd]
    w, V = np.linalg.eigh(Hk[np.ix_(sel, sel)])
    assert w[1] - w[0] > 1e-8   # a unique ground state
    full = np.zeros(dL * dR)
    full[sel] = V[:, 0]
    lam_k = np.sort(np.linalg.svd(full.reshape(dL, dR), compute_uv=False) ** 2)[::-1]
    s = O.Sector(m, nu, nd)
    e0, g = O.ground_state(s, I.psi(seed, s.n))
    assert abs(e0 - w[0]) < 1e-11
    ref = O.entanglement(s, g, "spatial", mask)
    lam_o = np.sort(np.concatenate(ref["lam"]))[::-1]
    np.testing.assert_allclose(lam_o, lam_k[:len(lam_o)], atol=1e-11)
    assert np.all(lam_k[len(lam_o):] < 1e-11)
