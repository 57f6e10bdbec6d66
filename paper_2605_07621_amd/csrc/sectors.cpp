// Sector builder: subsystem bases with colex ranking, the block list of
// Eq. (2)-(3), the subsystem operators H_L, H_R, their diagonals, the
// diagonal cross-cut terms and the sector-changing cross terms, plus the
// tables of the Hubbard up/down kernel.  Host only (no HIP calls).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "ecut_internal.h"
#include "kernels.h"

namespace ecut {

static uint64_t g_binom[65][65];
static std::once_flag g_binom_once;

static void init_binom() {
    for (int n = 0; n <= 64; ++n) {
        g_binom[n][0] = 1;
        for (int k = 1; k <= 64; ++k)
            g_binom[n][k] = (n == 0) ? 0 : g_binom[n - 1][k - 1] + g_binom[n - 1][k];
    }
}

uint64_t binom(int n, int k) {
    std::call_once(g_binom_once, init_binom);
    if (n < 0 || k < 0 || k > n || n > 64) return 0;
    return g_binom[n][k];
}

int64_t colex_rank(uint64_t w) {
    int64_t r = 0;
    int j = 0;
    while (w) {
        int p = __builtin_ctzll(w);
        r += (int64_t)binom(p, j + 1);
        ++j;
        w &= w - 1;
    }
    return r;
}

uint64_t colex_unrank(int64_t idx, int k) {
    uint64_t w = 0;
    for (int j = k; j >= 1; --j) {
        int p = j - 1;
        while ((int64_t)binom(p + 1, j) <= idx) ++p;
        w |= 1ull << p;
        idx -= (int64_t)binom(p, j);
    }
    return w;
}

namespace {

struct Sub {
    int n = 0;                 // bits
    int cmin = 0, cmax = -1;   // counts held
    std::vector<int32_t> cbase;
    std::vector<uint32_t> words;
    // off-diagonal rows before merging: (col, val) per global word
    std::vector<std::vector<std::pair<int32_t, double>>> rows;
    std::vector<double> diag;

    void build(int nbits, int c0, int c1) {
        n = nbits;
        cmin = std::max(c0, 0);
        cmax = std::min(c1, nbits);
        cbase.clear();
        words.clear();
        for (int c = cmin; c <= cmax; ++c) {
            cbase.push_back((int32_t)words.size());
            int64_t cnt = (int64_t)binom(n, c);
            for (int64_t i = 0; i < cnt; ++i) words.push_back((uint32_t)colex_unrank(i, c));
        }
        rows.assign(words.size(), {});
        diag.assign(words.size(), 0.0);
    }
    bool has_count(int c) const { return c >= cmin && c <= cmax; }
    int32_t base(int c) const { return cbase[c - cmin]; }
    // global index of word w (its count must be held)
    int64_t gindex(uint32_t w) const { return base(__builtin_popcount(w)) + colex_rank(w); }

    void to_csr(std::vector<int32_t> &ptr, std::vector<int32_t> &col, std::vector<double> &val) {
        ptr.assign(words.size() + 1, 0);
        col.clear();
        val.clear();
        for (size_t g = 0; g < words.size(); ++g) {
            auto &r = rows[g];
            std::sort(r.begin(), r.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            for (size_t e = 0; e < r.size(); ++e) {
                if (!col.empty() && (int64_t)col.size() > ptr[g] && col.back() == r[e].first) {
                    val.back() += r[e].second;
                } else {
                    col.push_back(r[e].first);
                    val.push_back(r[e].second);
                }
            }
            ptr[g + 1] = (int32_t)col.size();
        }
        rows.clear();
        rows.shrink_to_fit();
    }

    // map of the global word index under "clear bit b" (del) or "set bit b"
    // (ins): rank inside the target count, or -1.
    void bit_map(int b, bool ins, std::vector<int32_t> &out) const {
        for (size_t g = 0; g < words.size(); ++g) {
            uint32_t w = words[g];
            bool set = (w >> b) & 1u;
            int c = __builtin_popcount(w);
            int32_t v = -1;
            if (ins && !set && has_count(c + 1)) v = (int32_t)colex_rank(w | (1u << b));
            if (!ins && set && has_count(c - 1)) v = (int32_t)colex_rank(w & ~(1u << b));
            out.push_back(v);
        }
    }
};

inline double sz(uint32_t w, int b) { return ((w >> b) & 1u) ? 0.5 : -0.5; }

// Hop of a spinless fermion species between local sites i and j on word w:
// returns false if it vanishes, else the new word and the Jordan-Wigner sign
// (-1)^(number of particles strictly between i and j).
inline bool fermion_hop(uint32_t w, int i, int j, uint32_t &w2, int &sign) {
    bool ni = (w >> i) & 1u, nj = (w >> j) & 1u;
    if (ni == nj) return false;
    int lo = std::min(i, j), hi = std::max(i, j);
    uint32_t between = (hi - lo > 1) ? (((1u << (hi - lo - 1)) - 1u) << (lo + 1)) : 0u;
    sign = (__builtin_popcount(w & between) & 1) ? -1 : 1;
    w2 = w ^ ((1u << i) | (1u << j));
    return true;
}

}  // namespace

static void build_hub_tables(ecut_sectors *s, const ecut_model_desc *m);
static void build_spin_tables(ecut_sectors *s);
static void fold_cross_diagonal(ecut_sectors *s);
static void build_two_pass_tables(ecut_sectors *s, int lbits, const std::vector<uint32_t> &rbetw);
static int inversions(uint32_t w, int n);
static void build_hubseg_tables(ecut_sectors *s);
static void make_rank_tables(ecut_sectors *s);
static void build_hubrow_tables(ecut_sectors *s, const ecut_model_desc *m);
static void build_hub6_tables(ecut_sectors *s, const ecut_model_desc *m);
void make_row_order(const ecut_sectors *s, int order, std::vector<int32_t> &out);
void make_hub_item_order(const ecut_sectors *s, int order, std::vector<HubItem> &out);

// Hubbard model with a spatial cut (the paper's Fig. 1(b)): L = the sites
// of left_mask, R = the others.  A subsystem word is (up << n) | dn over the
// subsystem's n sites in site order; the bipartite basis state |l, r> is the
// ordered product of the creation operators of l's occupied modes (up modes
// by site, then down modes by site), then r's, on the vacuum.  Blocks are
// (N_up_L, N_dn_L) in lexicographic order; rows (columns) are the L (R)
// words of the block's numbers in increasing integer order, so the rank of
// a word inside its group is rank(up) * C(n, N_dn) + rank(dn).
//  - hops inside L or inside R: CSR rows of H_L, H_R with the sign of the
//    same-spin particles of that part strictly between the two sites;
//  - U_i and V_b inside a part: the part's diagonal;
//  - hops across the cut: per bond and spin the two directions of
//    -t (c+_i c_j + h.c.), i in L: gathering (l, r) from (l - i, r + j) the
//    sign is (-1)^(N_L(l) - 1 + occ_before_i(l)) * (-1)^(occ_before_j(r)),
//    from (l + i, r - j) it is (-1)^(N_L(l) + occ_before_i(l)) *
//    (-1)^(occ_before_j(r)) (the right operator passes every left
//    particle; occ_before counts the part's occupied modes before the mode
//    in the part's order);
//  - V_b across the cut: a diagonal cross term of the two site densities.
static ecut_status build_hubbard_spatial(const ecut_model_desc *m, const ecut_cut_desc *c, ecut_qnum q,
                                         ecut_sectors *s, Sub &L, Sub &R) {
    const int S = m->n_sites;
    if (S > 32) return fail(ECUT_EUNSUPPORTED, "Hubbard models up to 32 sites");
    if (m->n_bonds > 0 && !m->t) return fail(ECUT_EINVAL, "Hubbard model needs t");
    const uint64_t full = S == 64 ? ~0ull : ((1ull << S) - 1);
    if (c->left_mask & ~full) return fail(ECUT_EINVAL, "left_mask names sites beyond n_sites");
    if (q.n_up < 0 || q.n_up > S || q.n_dn < 0 || q.n_dn > S) return fail(ECUT_EINVAL, "particle numbers outside 0..n_sites");
    s->lsites.clear();
    s->rsites.clear();
    for (int i = 0; i < S; ++i) ((c->left_mask >> i) & 1u ? s->lsites : s->rsites).push_back(i);
    const int nL = (int)s->lsites.size(), nR = (int)s->rsites.size();
    if (nL > 16 || nR > 16) return fail(ECUT_EUNSUPPORTED, "spatial Hubbard cuts need at most 16 sites on each side");
    std::vector<int> side(S), loc(S);
    for (int k = 0; k < nL; ++k) { side[s->lsites[k]] = 0; loc[s->lsites[k]] = k; }
    for (int k = 0; k < nR; ++k) { side[s->rsites[k]] = 1; loc[s->rsites[k]] = k; }
    const int Nu = q.n_up, Nd = q.n_dn;
    // groups of subsystem words by (up, down) numbers
    auto groups = [](Sub &X, int n, int a0, int a1, int b0, int b1, std::map<std::pair<int, int>, int32_t> &base) {
        X.n = 2 * n;
        X.words.clear();
        for (int a = a0; a <= a1; ++a)
            for (int b = b0; b <= b1; ++b) {
                base[{a, b}] = (int32_t)X.words.size();
                const int64_t nu = (int64_t)binom(n, a), nd = (int64_t)binom(n, b);
                for (int64_t i = 0; i < nu; ++i)
                    for (int64_t k = 0; k < nd; ++k)
                        X.words.push_back(((uint32_t)colex_unrank(i, a) << n) | (uint32_t)colex_unrank(k, b));
            }
        X.rows.assign(X.words.size(), {});
        X.diag.assign(X.words.size(), 0.0);
    };
    const int la0 = std::max(0, Nu - nR), la1 = std::min(nL, Nu), lb0 = std::max(0, Nd - nR), lb1 = std::min(nL, Nd);
    if (la0 > la1 || lb0 > lb1) return fail(ECUT_EINVAL, "empty sector");
    std::map<std::pair<int, int>, int32_t> lbase, rbase;
    groups(L, nL, la0, la1, lb0, lb1, lbase);
    groups(R, nR, Nu - la1, Nu - la0, Nd - lb1, Nd - lb0, rbase);
    L.cmin = R.cmin = 0;
    L.cmax = R.cmax = -1;
    // blocks
    s->blocks.clear();
    std::map<std::pair<int, int>, int32_t> bidx;
    int64_t off = 0;
    for (int a = la0; a <= la1; ++a)
        for (int b = lb0; b <= lb1; ++b) {
            BlockDev B{};
            B.offset = off;
            B.q_l = a;
            B.q_l2 = b;
            B.q_r = Nu - a;
            B.q_r2 = Nd - b;
            B.d_l = (int32_t)(binom(nL, a) * binom(nL, b));
            B.d_r = (int32_t)(binom(nR, Nu - a) * binom(nR, Nd - b));
            B.lbase = lbase[{a, b}];
            B.rbase = rbase[{Nu - a, Nd - b}];
            bidx[{a, b}] = (int32_t)s->blocks.size();
            off += (int64_t)B.d_l * B.d_r;
            s->blocks.push_back(B);
        }
    for (BlockDev &B : s->blocks) {
        auto nb = [&](int a, int b) {
            auto it = bidx.find({a, b});
            return it == bidx.end() ? -1 : it->second;
        };
        B.blk_lminus = nb(B.q_l - 1, B.q_l2);
        B.blk_lplus = nb(B.q_l + 1, B.q_l2);
        B.blk_l2minus = nb(B.q_l, B.q_l2 - 1);
        B.blk_l2plus = nb(B.q_l, B.q_l2 + 1);
    }
    s->dim = off;
    // rank of a subsystem word inside its (up, down) group
    auto grank = [](uint32_t w, int n) -> int32_t {
        const uint32_t dn = w & ((1u << n) - 1u), up = w >> n;
        return (int32_t)(colex_rank(up) * (int64_t)binom(n, __builtin_popcount(dn)) + colex_rank(dn));
    };
    // occupied modes of a part before mode (spin, k) in the part's order
    auto occ_before = [](uint32_t w, int n, int spin, int k) -> int {
        const uint32_t dn = w & ((1u << n) - 1u), up = w >> n;
        const uint32_t below = (1u << k) - 1u;
        return spin == 0 ? __builtin_popcount(up & below) : __builtin_popcount(up) + __builtin_popcount(dn & below);
    };
    auto density = [](uint32_t w, int n, int k) { return (int)((w >> (n + k)) & 1u) + (int)((w >> k) & 1u); };
    // operators inside the two parts
    for (int part = 0; part < 2; ++part) {
        Sub &X = part == 0 ? L : R;
        const int n = part == 0 ? nL : nR;
        for (size_t g = 0; g < X.words.size(); ++g) {
            const uint32_t w = X.words[g];
            for (int k = 0; k < n; ++k) {
                const int site = part == 0 ? s->lsites[k] : s->rsites[k];
                if (m->u && ((w >> (n + k)) & 1u) && ((w >> k) & 1u)) X.diag[g] += m->u[site];
            }
        }
        for (int b = 0; b < m->n_bonds; ++b) {
            const int i = m->bond_i[b], j = m->bond_j[b];
            if (side[i] != part || side[j] != part) continue;
            const int li = loc[i], lj = loc[j];
            const double t = m->t[b], v = m->v ? m->v[b] : 0.0;
            for (size_t g = 0; g < X.words.size(); ++g) {
                const uint32_t w = X.words[g];
                if (v != 0.0) X.diag[g] += v * density(w, n, li) * density(w, n, lj);
                if (t == 0.0) continue;
                const uint32_t dn = w & ((1u << n) - 1u), up = w >> n;
                uint32_t w2;
                int sg;
                if (fermion_hop(up, li, lj, w2, sg)) X.rows[g].push_back({grank((w2 << n) | dn, n), -t * sg});
                if (fermion_hop(dn, li, lj, w2, sg)) X.rows[g].push_back({grank((up << n) | w2, n), -t * sg});
            }
        }
    }
    // across the cut
    s->xdiag.clear();
    s->xbond.clear();
    s->maps.clear();
    s->n_cut_bonds = 0;
    auto has_group = [](const std::map<std::pair<int, int>, int32_t> &base, uint32_t w, int n) {
        return base.count({__builtin_popcount(w >> n), __builtin_popcount(w & ((1u << n) - 1u))}) != 0;
    };
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_i[b], j = m->bond_j[b];
        if (side[i] == side[j]) continue;
        if (side[i] == 1) std::swap(i, j);   // i in L, j in R
        ++s->n_cut_bonds;
        const int li = loc[i], rj = loc[j];
        const double v = m->v ? m->v[b] : 0.0;
        if (v != 0.0) s->xdiag.push_back(XDiagDev{nL + li, nR + rj, 0, li, rj, 0, v});
        if (m->t[b] == 0.0) continue;
        for (int spin = 0; spin < 2; ++spin) {
            XBondDev X{};
            X.li = spin == 0 ? nL + li : li;
            X.rj = spin == 0 ? nR + rj : rj;
            X.coef = -m->t[b];
            X.label = spin;
            X.fermion = 1;
            const uint32_t lbit = 1u << X.li, rbit = 1u << X.rj;
            X.lmap_del = (int32_t)s->maps.size();
            for (uint32_t w : L.words) {   // target has mode i: source l - i
                int32_t e = -1;
                if ((w & lbit) && has_group(lbase, w ^ lbit, nL)) {
                    const int par = __builtin_popcount(w) - 1 + occ_before(w, nL, spin, li);
                    e = (grank(w ^ lbit, nL) << 1) | (par & 1);
                }
                s->maps.push_back(e);
            }
            X.lmap_ins = (int32_t)s->maps.size();
            for (uint32_t w : L.words) {   // target lacks mode i: source l + i
                int32_t e = -1;
                if (!(w & lbit) && has_group(lbase, w | lbit, nL)) {
                    const int par = __builtin_popcount(w) + occ_before(w, nL, spin, li);
                    e = (grank(w | lbit, nL) << 1) | (par & 1);
                }
                s->maps.push_back(e);
            }
            X.rmap_ins = (int32_t)s->maps.size();
            for (uint32_t w : R.words) {   // source r + j
                int32_t e = -1;
                if (!(w & rbit) && has_group(rbase, w | rbit, nR))
                    e = (grank(w | rbit, nR) << 1) | (occ_before(w, nR, spin, rj) & 1);
                s->maps.push_back(e);
            }
            X.rmap_del = (int32_t)s->maps.size();
            for (uint32_t w : R.words) {   // source r - j
                int32_t e = -1;
                if ((w & rbit) && has_group(rbase, w ^ rbit, nR))
                    e = (grank(w ^ rbit, nR) << 1) | (occ_before(w, nR, spin, rj) & 1);
                s->maps.push_back(e);
            }
            s->xbond.push_back(X);
        }
    }
    // the cross terms of one left mode together (the two-pass kernels stage
    // the one source row of a left mode once for all its terms)
    std::stable_sort(s->xbond.begin(), s->xbond.end(), [](const XBondDev &a, const XBondDev &b) { return a.li < b.li; });
    // hops inside R as right terms of the two-pass kernels: the two bits of
    // the hop in the right word, the bits strictly between them (the fermion
    // sign), the value -t
    s->spin_fmask.clear();
    s->spin_fcoef.clear();
    s->sp_rbetw.clear();
    for (int b = 0; b < m->n_bonds; ++b) {
        const int i = m->bond_i[b], j = m->bond_j[b];
        if (side[i] != 1 || side[j] != 1 || m->t[b] == 0.0) continue;
        const int lo = std::min(loc[i], loc[j]), hi = std::max(loc[i], loc[j]);
        for (int spin = 0; spin < 2; ++spin) {
            const int o = spin == 0 ? nR : 0;
            s->spin_fmask.push_back((1u << (o + lo)) | (1u << (o + hi)));
            s->sp_rbetw.push_back(((1u << (o + hi)) - 1u) & ~((1u << (o + lo + 1)) - 1u));
            s->spin_fcoef.push_back(-m->t[b]);
        }
    }
    s->hub_spatial = true;
    return ECUT_OK;
}

ecut_status build_host(const ecut_model_desc *m, const ecut_cut_desc *c, ecut_qnum q, ecut_sectors *s) {
    if (!m || !c) return fail(ECUT_EINVAL, "null model or cut");
    if (m->reserved != 0 || c->reserved != 0) return fail(ECUT_EINVAL, "reserved fields must be 0");
    if (m->kind != ECUT_SPIN_HALF && m->kind != ECUT_HUBBARD) return fail(ECUT_EINVAL, "unknown model kind");
    if (m->n_sites <= 0) return fail(ECUT_EINVAL, "n_sites must be positive");
    if (m->n_bonds < 0 || (m->n_bonds > 0 && (!m->bond_i || !m->bond_j)))
        return fail(ECUT_EINVAL, "bad bond arrays");
    for (int b = 0; b < m->n_bonds; ++b) {
        int i = m->bond_i[b], j = m->bond_j[b];
        if (i < 0 || j < 0 || i >= m->n_sites || j >= m->n_sites || i == j)
            return fail(ECUT_EINVAL, "bond " + std::to_string(b) + " has invalid end points");
    }
    s->kind = m->kind;
    s->cut_kind = c->kind;
    s->n_sites = m->n_sites;
    s->left_mask = c->left_mask;
    s->n_up = q.n_up;
    s->n_dn = q.n_dn;

    Sub L, R;
    if (m->kind == ECUT_SPIN_HALF) {
        if (c->kind != ECUT_CUT_SPATIAL) return fail(ECUT_EINVAL, "spin models take a spatial cut");
        if (m->n_sites > 64) return fail(ECUT_EUNSUPPORTED, "spin models up to 64 sites");
        if (m->n_bonds > 0 && (!m->jxy || !m->jz)) return fail(ECUT_EINVAL, "spin model needs jxy and jz");
        uint64_t full = (m->n_sites == 64) ? ~0ull : ((1ull << m->n_sites) - 1);
        if (c->left_mask & ~full) return fail(ECUT_EINVAL, "left_mask names sites beyond n_sites");
        if (q.n_up < 0 || q.n_up > m->n_sites) return fail(ECUT_EINVAL, "n_up outside 0..n_sites");
        s->lsites.clear();
        s->rsites.clear();
        for (int i = 0; i < m->n_sites; ++i) ((c->left_mask >> i) & 1u ? s->lsites : s->rsites).push_back(i);
        int nL = (int)s->lsites.size(), nR = (int)s->rsites.size();
        if (nL > 32 || nR > 32) return fail(ECUT_EUNSUPPORTED, "each side of the cut may hold at most 32 sites");
        int qmin = std::max(0, q.n_up - nR), qmax = std::min(nL, q.n_up);
        L.build(nL, qmin, qmax);
        R.build(nR, q.n_up - qmax, q.n_up - qmin);
        std::vector<int> side(m->n_sites), loc(m->n_sites);
        for (int k = 0; k < nL; ++k) { side[s->lsites[k]] = 0; loc[s->lsites[k]] = k; }
        for (int k = 0; k < nR; ++k) { side[s->rsites[k]] = 1; loc[s->rsites[k]] = k; }
        // blocks
        s->blocks.clear();
        int64_t off = 0;
        for (int ql = qmin; ql <= qmax; ++ql) {
            BlockDev B{};
            B.offset = off;
            B.q_l = ql;
            B.q_r = q.n_up - ql;
            B.d_l = (int32_t)binom(nL, ql);
            B.d_r = (int32_t)binom(nR, B.q_r);
            B.lbase = L.base(ql);
            B.rbase = R.base(B.q_r);
            B.blk_lminus = ql > qmin ? (int32_t)s->blocks.size() - 1 : -1;
            B.blk_lplus = ql < qmax ? (int32_t)s->blocks.size() + 1 : -1;
            B.blk_l2minus = B.blk_l2plus = -1;
            off += (int64_t)B.d_l * B.d_r;
            s->blocks.push_back(B);
        }
        s->dim = off;
        // operators
        std::map<int, int32_t> lmaps_del, lmaps_ins, rmaps_del, rmaps_ins;
        s->xdiag.clear();
        s->xbond.clear();
        s->maps.clear();
        s->n_cut_bonds = 0;
        auto map_for = [&](Sub &S, std::map<int, int32_t> &cache, int bit, bool ins) {
            auto it = cache.find(bit);
            if (it != cache.end()) return it->second;
            int32_t o = (int32_t)s->maps.size();
            S.bit_map(bit, ins, s->maps);
            cache[bit] = o;
            return o;
        };
        for (int b = 0; b < m->n_bonds; ++b) {
            int i = m->bond_i[b], j = m->bond_j[b];
            double jxy = m->jxy[b], jz = m->jz[b];
            if (side[i] == side[j]) {
                Sub &S = side[i] == 0 ? L : R;
                int bi = loc[i], bj = loc[j];
                for (size_t g = 0; g < S.words.size(); ++g) {
                    uint32_t w = S.words[g];
                    S.diag[g] += jz * sz(w, bi) * sz(w, bj);
                    if (jxy != 0.0 && (((w >> bi) ^ (w >> bj)) & 1u)) {
                        uint32_t w2 = w ^ ((1u << bi) | (1u << bj));
                        S.rows[g].push_back({(int32_t)colex_rank(w2), 0.5 * jxy});
                    }
                }
                if (side[i] == 1 && jxy != 0.0) {
                    s->spin_fmask.push_back((1u << bi) | (1u << bj));
                    s->spin_fcoef.push_back(0.5 * jxy);
                }
            } else {
                ++s->n_cut_bonds;
                int li = side[i] == 0 ? loc[i] : loc[j];
                int rj = side[i] == 0 ? loc[j] : loc[i];
                if (jz != 0.0) s->xdiag.push_back(XDiagDev{li, rj, 1, -1, -1, 0, jz});
                if (jxy != 0.0) {
                    XBondDev X{};
                    X.li = li;
                    X.rj = rj;
                    X.coef = 0.5 * jxy;
                    X.lmap_del = map_for(L, lmaps_del, li, false);
                    X.lmap_ins = map_for(L, lmaps_ins, li, true);
                    X.rmap_del = map_for(R, rmaps_del, rj, false);
                    X.rmap_ins = map_for(R, rmaps_ins, rj, true);
                    s->xbond.push_back(X);
                }
            }
        }
        // cross bonds grouped by their left site: the spin kernel stages the
        // one source row of a left site once for all its bonds
        std::stable_sort(s->xbond.begin(), s->xbond.end(),
                         [](const XBondDev &a, const XBondDev &b) { return a.li < b.li; });
    } else if (c->kind == ECUT_CUT_SPATIAL) {
        ecut_status st = build_hubbard_spatial(m, c, q, s, L, R);
        if (st != ECUT_OK) return st;
    } else {
        if (c->kind != ECUT_CUT_UPDN) return fail(ECUT_EINVAL, "unknown cut kind");
        if (m->n_sites > 32) return fail(ECUT_EUNSUPPORTED, "Hubbard models up to 32 sites");
        if (m->v)
            for (int b = 0; b < m->n_bonds; ++b)
                if (m->v[b] != 0.0)
                    return fail(ECUT_EUNSUPPORTED, "the bond interaction V is built for the spatial cut only");
        if (m->n_bonds > 0 && !m->t) return fail(ECUT_EINVAL, "Hubbard model needs t");
        int Ls = m->n_sites;
        if (q.n_up < 0 || q.n_up > Ls || q.n_dn < 0 || q.n_dn > Ls)
            return fail(ECUT_EINVAL, "particle numbers outside 0..n_sites");
        s->lsites.clear();
        for (int i = 0; i < Ls; ++i) s->lsites.push_back(i);
        s->rsites = s->lsites;
        L.build(Ls, q.n_up, q.n_up);
        R.build(Ls, q.n_dn, q.n_dn);
        BlockDev B{};
        B.offset = 0;
        B.q_l = q.n_up;
        B.q_r = q.n_dn;
        B.d_l = (int32_t)binom(Ls, q.n_up);
        B.d_r = (int32_t)binom(Ls, q.n_dn);
        B.lbase = 0;
        B.rbase = 0;
        B.blk_lminus = B.blk_lplus = B.blk_l2minus = B.blk_l2plus = -1;
        s->blocks.assign(1, B);
        s->dim = (int64_t)B.d_l * B.d_r;
        for (Sub *S : {&L, &R}) {
            for (int b = 0; b < m->n_bonds; ++b) {
                double t = m->t[b];
                if (t == 0.0) continue;
                int i = m->bond_i[b], j = m->bond_j[b];
                for (size_t g = 0; g < S->words.size(); ++g) {
                    uint32_t w2;
                    int sg;
                    if (fermion_hop(S->words[g], i, j, w2, sg))
                        S->rows[g].push_back({(int32_t)colex_rank(w2), -t * sg});
                }
            }
        }
        s->xdiag.clear();
        s->xbond.clear();
        s->maps.clear();
        s->n_cut_bonds = 0;
        if (m->u)
            for (int i = 0; i < Ls; ++i)
                if (m->u[i] != 0.0) s->xdiag.push_back(XDiagDev{i, i, 0, -1, -1, 0, m->u[i]});
    }

    s->lcmin = L.cmin;
    s->lcmax = L.cmax;
    s->rcmin = R.cmin;
    s->rcmax = R.cmax;
    s->lcbase = L.cbase;
    s->rcbase = R.cbase;
    s->lwords = L.words;
    s->rwords = R.words;
    s->diag_l = L.diag;
    s->diag_r = R.diag;
    L.to_csr(s->hl_ptr, s->hl_col, s->hl_val);
    R.to_csr(s->hr_ptr, s->hr_col, s->hr_val);

    s->max_d_r = 0;
    double sw2 = 0.0;
    for (auto &B : s->blocks) {
        s->max_d_r = std::max(s->max_d_r, B.d_r);
        double w = (double)B.d_l * (double)B.d_r / (double)s->dim;
        sw2 += w * w;
    }
    s->n_eff = sw2 > 0 ? 1.0 / sw2 : 0.0;

    // default work items of the generic row kernel: row tiles of about
    // `tile` elements (at least one row), largest first
    const int64_t tile = std::max<int64_t>(s->max_d_r, 2048);
    s->items.clear();
    for (int b = 0; b < (int)s->blocks.size(); ++b) {
        const BlockDev &B = s->blocks[b];
        int32_t rpt = (int32_t)std::max<int64_t>(1, std::min<int64_t>(B.d_l, tile / std::max(B.d_r, 1)));
        for (int32_t r0 = 0; r0 < B.d_l; r0 += rpt)
            s->items.push_back(ItemDev{0, b, r0, std::min(B.d_l, r0 + rpt), 0, 0});
    }
    std::stable_sort(s->items.begin(), s->items.end(), [&](const ItemDev &a, const ItemDev &b) {
        int64_t wa = (int64_t)(a.row1 - a.row0) * s->blocks[a.block].d_r;
        int64_t wb = (int64_t)(b.row1 - b.row0) * s->blocks[b.block].d_r;
        return wa > wb;
    });
    for (size_t k = 0; k < s->items.size(); ++k) s->items[k].slot = (int32_t)k;
    s->items_cap = s->items.size();
    s->item_slots = s->item_slots_cap = (int32_t)s->items.size();

    s->hub_ok = false;
    s->kernel = 2;
    fold_cross_diagonal(s);
    build_spin_tables(s);
    if (s->hub_spatial) {
        // two-pass kernels over one-row items (every row its own item)
        s->generic_items = s->items;
        make_rank_tables(s);
        build_two_pass_tables(s, 2 * (int)s->lsites.size(), s->sp_rbetw);
        size_t rows = 0;
        for (const BlockDev &B : s->blocks) rows += (size_t)B.d_l;
        s->items_cap = std::max(s->items_cap, rows);
        s->item_slots_cap = std::max<int32_t>(s->item_slots_cap, (int32_t)rows);
    }
    if (s->kind == ECUT_HUBBARD && s->cut_kind == ECUT_CUT_UPDN) build_hub_tables(s, m);
    return ECUT_OK;
}

// Tables of the Hubbard up/down kernel.  Down words of n_r bits are split at
// h = n_r / 2 into lo (bits < h) and hi (bits >= h); with the colex order of
// the fixed-count down basis, the column of (hi, lo) is seg_off[hi] +
// lo_rank[lo] because all words sharing hi are contiguous and ordered by lo.
static void build_hub_tables(ecut_sectors *s, const ecut_model_desc *m) {
    const BlockDev &B = s->blocks[0];
    int n = s->n_sites;
    int c = B.q_r;
    // the kernel holds a full row plus these tables in LDS
    if (n > 20 || (int64_t)B.d_r * 8 > 120 * 1024 || B.d_r < 1) return;
    int h = n / 2;
    int nlo = 1 << h, nhi = 1 << (n - h);
    ecut::HubDev &H = s->hub;
    H = ecut::HubDev{};
    H.n_r = n;
    H.h = h;
    // coefficient table: distinct -t_b values
    std::vector<double> coef;
    std::vector<int> bcoef(m->n_bonds, -1);
    for (int b = 0; b < m->n_bonds; ++b) {
        double v = -m->t[b];
        if (m->t[b] == 0.0) continue;
        auto it = std::find(coef.begin(), coef.end(), v);
        if (it == coef.end()) { coef.push_back(v); bcoef[b] = (int)coef.size() - 1; }
        else bcoef[b] = (int)(it - coef.begin());
    }
    if (coef.size() > 255) return;
    H.n_coef = (int32_t)coef.size();
    H.uniform_t = coef.size() <= 1 ? 1 : 0;
    H.hop0 = coef.empty() ? 0.0 : coef[0];
    // lo/hi neighbour lists
    std::vector<std::vector<int32_t>> lo_l(nlo), hi_l(nhi);
    std::vector<int32_t> lo_rank(nlo), seg_off(nhi, -1);
    for (int v = 0; v < nlo; ++v) lo_rank[v] = (int32_t)ecut::colex_rank((uint64_t)v);
    {
        // class-major column order: segments grouped by popc(hi), then by hi;
        // every class (all segments of one popc(hi)) is one contiguous run of
        // columns, so a class tile of a row is contiguous memory
        int32_t acc = 0;
        for (int kh = 0; kh <= n - h; ++kh)
            for (int u = 0; u < nhi; ++u) {
                if (__builtin_popcount(u) != kh) continue;
                int k = c - kh;
                if (k < 0 || k > h) continue;
                seg_off[u] = acc;
                acc += (int32_t)ecut::binom(h, k);
            }
        if (acc != B.d_r) return;   // cannot happen; keeps the kernel honest
    }
    auto pack = [](int32_t delta, int neg, int ci) { return (int32_t)(((uint32_t)delta << 9) | (uint32_t)(neg << 8) | (uint32_t)ci); };
    std::vector<int32_t> xb;
    for (int b = 0; b < m->n_bonds; ++b) {
        if (bcoef[b] < 0) continue;
        int i = m->bond_i[b], j = m->bond_j[b];
        if (i < h && j < h) {
            for (int v = 0; v < nlo; ++v) {
                uint32_t w2;
                int sg;
                if (fermion_hop((uint32_t)v, i, j, w2, sg))
                    lo_l[v].push_back(pack(lo_rank[w2] - lo_rank[v], sg < 0, bcoef[b]));
            }
        } else if (i >= h && j >= h) {
            for (int u = 0; u < nhi; ++u) {
                uint32_t w2;
                int sg;
                if (seg_off[u] >= 0 && fermion_hop((uint32_t)u, i - h, j - h, w2, sg))
                    hi_l[u].push_back(pack(seg_off[w2] - seg_off[u], sg < 0, bcoef[b]));
            }
        } else {
            int lb = i < h ? i : j, hb = (i < h ? j : i) - h;
            xb.push_back(lb);
            xb.push_back(hb);
            xb.push_back(bcoef[b]);
            xb.push_back(0);
        }
    }
    size_t ls = 1, hs = 1;
    for (auto &v : lo_l) ls = std::max(ls, v.size());
    for (auto &v : hi_l) hs = std::max(hs, v.size());
    {
        // the whole LDS image (row, words, tables) must fit 160 KiB
        auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
        size_t lds = al((size_t)B.d_r * 8) + al((size_t)B.d_r * (n <= 16 ? 2 : 4)) + 2 * al((size_t)nlo * 4) +
                     al((size_t)nlo * ls * 4) + 2 * al((size_t)nhi * 4) + al((size_t)nhi * hs * 4) +
                     al(std::max<size_t>(coef.size(), 1) * 8) + 3 * 256 * 8 + 1024;
        if (lds > 160 * 1024) return;
    }
    H.lo_stride = (int32_t)ls;
    H.hi_stride = (int32_t)hs;
    H.n_xb = (int32_t)(xb.size() / 4);
    s->hub_lo_cnt.assign(nlo, 0);
    s->hub_lo_ent.assign((size_t)nlo * ls, 0);
    s->hub_hi_cnt.assign(nhi, 0);
    s->hub_hi_ent.assign((size_t)nhi * hs, 0);
    for (int v = 0; v < nlo; ++v) {
        s->hub_lo_cnt[v] = (int32_t)lo_l[v].size();
        std::copy(lo_l[v].begin(), lo_l[v].end(), s->hub_lo_ent.begin() + (size_t)v * ls);
    }
    for (int u = 0; u < nhi; ++u) {
        s->hub_hi_cnt[u] = (int32_t)hi_l[u].size();
        std::copy(hi_l[u].begin(), hi_l[u].end(), s->hub_hi_ent.begin() + (size_t)u * hs);
    }
    s->hub_lo_rank = lo_rank;
    s->hub_seg_off = seg_off;
    s->hub_xb = xb;
    s->hub_coef = coef.empty() ? std::vector<double>{0.0} : coef;
    s->hub_u.assign(n, 0.0);
    if (m->u)
        for (int i = 0; i < n; ++i) s->hub_u[i] = m->u[i];
    H.uniform_u = 1;
    H.u0 = s->hub_u[0];
    for (int i = 1; i < n; ++i)
        if (s->hub_u[i] != H.u0) H.uniform_u = 0;
    // canonical (colex) rank of a down word -> its column; down words by column
    s->hub_col_of_rank.assign(B.d_r, 0);
    s->hub_rw32.assign(B.d_r, 0);
    s->hub_rw16.clear();
    if (n <= 16) s->hub_rw16.assign(B.d_r, 0);
    for (int32_t r = 0; r < B.d_r; ++r) {
        const uint32_t w = s->rwords[B.rbase + r];
        const int32_t col = seg_off[w >> h] + lo_rank[w & ((1u << h) - 1u)];
        s->hub_col_of_rank[r] = col;
        s->hub_rw32[col] = w;
        if (n <= 16) s->hub_rw16[col] = (uint16_t)w;
    }
    build_hubrow_tables(s, m);
    build_hub6_tables(s, m);
    make_row_order(s, 1, s->level_rows);
    if (s->hub6_ok) processing_csr(s, s->level_rows, s->h6_pptr, s->h6_pcol, s->h6_pval);
    make_row_order(s, 0, s->row_order);

    // ---- class tiles of the down basis
    {
        const int nh = n - h;
        std::vector<std::vector<int32_t>> his(nh + 1);
        for (int u = 0; u < nhi; ++u) his[__builtin_popcount(u)].push_back(u);
        struct Cls {
            int k, L, nseg;
            std::vector<int32_t> segcol, hiw, low;
            std::vector<std::vector<int32_t>> hient, loent;
        };
        std::vector<Cls> cl;
        for (int k = 0; k <= nh; ++k) {
            const int lc = c - k;
            if (lc < 0 || lc > h) continue;
            Cls C;
            C.k = k;
            C.L = (int)ecut::binom(h, lc);
            C.nseg = (int)his[k].size();
            std::vector<int32_t> segidx(nhi, -1);
            for (int si = 0; si < C.nseg; ++si) {
                const int u = his[k][si];
                segidx[u] = si;
                C.hiw.push_back(u);
                C.segcol.push_back(seg_off[u]);
            }
            C.hient.resize(C.nseg);
            for (int v = 0; v < nlo; ++v)
                if (__builtin_popcount(v) == lc) C.low.push_back(v);
            C.loent.resize(C.L);
            for (int b = 0; b < m->n_bonds; ++b) {
                if (bcoef[b] < 0) continue;
                const int i = m->bond_i[b], j = m->bond_j[b];
                if (i >= h && j >= h) {
                    for (int si = 0; si < C.nseg; ++si) {
                        uint32_t w2;
                        int sg;
                        if (fermion_hop((uint32_t)C.hiw[si], i - h, j - h, w2, sg))
                            C.hient[si].push_back(pack(segidx[w2] - si, sg < 0, bcoef[b]));
                    }
                } else if (i < h && j < h) {
                    for (int jj = 0; jj < C.L; ++jj) {
                        uint32_t w2;
                        int sg;
                        if (fermion_hop((uint32_t)C.low[jj], i, j, w2, sg))
                            C.loent[jj].push_back(pack(lo_rank[w2] - jj, sg < 0, bcoef[b]));
                    }
                }
            }
            cl.push_back(std::move(C));
        }
        size_t hs2 = 1, ls2 = 1;
        for (auto &C : cl) {
            for (auto &v : C.hient) hs2 = std::max(hs2, v.size());
            for (auto &v : C.loent) ls2 = std::max(ls2, v.size());
        }
        // rows per item: the padded tile (row stride L + 1 in the fast
        // kernel) of every class stays within the largest one-row class tile,
        // so one-column classes do not double the LDS of a work group
        int tile_pad = 2048;
        for (auto &C : cl) tile_pad = std::max(tile_pad, C.nseg * (C.L + 1));
        s->hc_cls.clear();
        s->hc_segcol.clear();
        s->hc_hiw.clear();
        s->hc_hicnt.clear();
        s->hc_hient.clear();
        s->hc_low.clear();
        s->hc_locnt.clear();
        s->hc_loent.clear();
        s->hub_items.clear();
        int max_nseg = 1, max_tile = 1;
        for (size_t ci = 0; ci < cl.size(); ++ci) {
            Cls &C = cl[ci];
            const int seg_base = (int)s->hc_segcol.size(), lo_base = (int)s->hc_low.size();
            const int S = C.L * C.nseg;
            const int rpi = std::max(1, std::min(B.d_l, tile_pad / (C.nseg * (C.L + 1))));
            s->hc_cls.insert(s->hc_cls.end(), {C.L, C.nseg, seg_base, lo_base, rpi, S, C.k, 0});
            for (int si = 0; si < C.nseg; ++si) {
                s->hc_segcol.push_back(C.segcol[si]);
                s->hc_hiw.push_back(C.hiw[si]);
                s->hc_hicnt.push_back((int32_t)C.hient[si].size());
                for (size_t q = 0; q < hs2; ++q) s->hc_hient.push_back(q < C.hient[si].size() ? C.hient[si][q] : 0);
            }
            for (int jj = 0; jj < C.L; ++jj) {
                s->hc_low.push_back(C.low[jj]);
                s->hc_locnt.push_back((int32_t)C.loent[jj].size());
                for (size_t q = 0; q < ls2; ++q) s->hc_loent.push_back(q < C.loent[jj].size() ? C.loent[jj][q] : 0);
            }
            for (int32_t r0 = 0; r0 < B.d_l; r0 += rpi)
                s->hub_items.push_back(HubItem{r0, std::min(rpi, B.d_l - r0), (int32_t)ci, (int32_t)s->hub_items.size()});
            max_nseg = std::max(max_nseg, C.nseg);
            max_tile = std::max(max_tile, rpi * S);
        }
        // the class-tile kernel needs every class row to fit its thread block
        // (512 threads, at most 16 element passes) and the tile to fit LDS
        bool ok = true;
        for (size_t ci = 0; ci < cl.size(); ++ci) {
            const int L = s->hc_cls[8 * ci], nseg = s->hc_cls[8 * ci + 1], rpi = s->hc_cls[8 * ci + 4];
            const int per_pass = 512 / L;
            if (per_pass < 1 || (rpi * nseg + per_pass - 1) / per_pass > 16) ok = false;
        }
        if ((size_t)max_tile * 8 + (size_t)max_nseg * (12 + 4 * hs2) + 4 * (size_t)(nhi + nlo) + 4096 > 150 * 1024) ok = false;
        s->hub2_ok = ok;
        H.n_cls = (int32_t)cl.size();
        // ---- fast path: sign-free uniform hopping on both spins
        bool fast = ok && coef.size() == 1 && n <= 16 && H.uniform_u && xb.size() <= 4;
        if (fast && !xb.empty()) fast = xb[0] == h - 1 && xb[1] == 0;
        for (double v : s->hl_val) fast = fast && v == coef[0];
        for (auto &C : cl) {
            for (auto &v : C.hient) for (int en : v) fast = fast && !((en >> 8) & 1);
            for (auto &v : C.loent) for (int en : v) fast = fast && !((en >> 8) & 1);
        }
        if (fast) {
            s->h3_seginfo.clear();
            s->h3_loinfo.clear();
            s->h3_looff.clear();
            s->h3_hnb.clear();
            s->h3_hcnt.clear();
            const int hb = xb.empty() ? -1 : xb[1], lb = xb.empty() ? -1 : xb[0];
            int mt = 0;
            for (size_t ci = 0; ci < cl.size(); ++ci) {
                Cls &C = cl[ci];
                for (int si = 0; si < C.nseg; ++si) {
                    const int u = C.hiw[si];
                    int xcol = 0, xbit = 2;
                    if (hb >= 0) {
                        const int u2 = u ^ (1 << hb);
                        xbit = (u >> hb) & 1;
                        xcol = seg_off[u2] >= 0 ? seg_off[u2] : 0;
                    }
                    s->h3_seginfo.insert(s->h3_seginfo.end(), {C.segcol[si], u, xcol, xbit});
                    s->h3_hcnt.push_back((int32_t)C.hient[si].size());
                    for (size_t q = 0; q < hs2; ++q)
                        s->h3_hnb.push_back(q < C.hient[si].size() ? si + (C.hient[si][q] >> 9) : 0);
                }
                for (int jj = 0; jj < C.L; ++jj) {
                    const int v = C.low[jj];
                    int xlo = 0, xbit = 2;
                    if (lb >= 0) {
                        xbit = (v >> lb) & 1;
                        xlo = lo_rank[v ^ (1 << lb)];
                    }
                    s->h3_loinfo.insert(s->h3_loinfo.end(), {v, xlo, xbit, 0});
                    for (int q = 0; q < 8; ++q)
                        s->h3_looff.push_back(q < (int)C.loent[jj].size() ? (C.loent[jj][q] >> 9) : C.L - jj);
                    if (C.loent[jj].size() > 8) fast = false;
                }
                const int rpi = s->hc_cls[8 * ci + 4];
                mt = std::max(mt, rpi * C.nseg * (C.L + 1));
            }
            s->h3_hs = (int32_t)hs2;
            s->h3_max_tile = mt;
            // every item must fit HUB3_M element slots per thread of HUB3_THREADS
            int max_l = 0;
            for (size_t ci = 0; ci < cl.size(); ++ci) {
                const int L = s->hc_cls[8 * ci], nseg = s->hc_cls[8 * ci + 1], rpi = s->hc_cls[8 * ci + 4];
                max_l = std::max(max_l, L);
                const int per_pass = HUB3_THREADS / L;
                if (per_pass < 1 || (rpi * nseg + per_pass - 1) / per_pass > HUB3_M) fast = false;
                if ((int64_t)rpi * s->blocks[0].d_r > (1ll << 31) / 2) fast = false;
            }
            if ((size_t)mt * 8 + (size_t)max_nseg * (16 + 4 * hs2 + 4) + (size_t)max_l * 48 + 2048 > 150 * 1024) fast = false;
        }
        s->hub3_ok = fast;
        build_hubseg_tables(s);
        H.cls_lo_stride = (int32_t)ls2;
        H.cls_hi_stride = (int32_t)hs2;
        H.max_tile = max_tile;
        H.max_nseg = max_nseg;
        s->hub_items_cap = s->hub_items.size();
        for (int order = 6; order <= 8; ++order) {
            make_hub_item_order(s, order, s->hub_items_ord);
            s->hub_items_cap = std::max(s->hub_items_cap, s->hub_items_ord.size());
        }
        make_hub_item_order(s, 0, s->hub_items_ord);
    }
    s->hub_ok = true;
    s->kernel = 1;
}

// Tables of the segment-tile kernel (uniform, sign-free hopping, as the fast
// class-tile kernel).  The down side reuses that kernel's segment and
// low-word tables.  The up side is read off the up-hopping CSR: a hop that
// keeps the high half of the up word is a low-half hop inside the segment (a
// row offset), one that keeps the low half moves to the same row of a
// neighbour segment, any other is the crossing-bond hop (at most one per
// row).  Anything that does not fit this shape leaves the kernel off.
static void build_hubseg_tables(ecut_sectors *s) {
    s->hubseg_ok = false;
    s->hs_useg.clear();
    s->hs_uhnb.clear();
    s->hs_ulo.clear();
    s->hs_ucross.clear();
    s->hs_items.clear();
    if (!s->hub3_ok) return;
    const BlockDev &B = s->blocks[0];
    if (B.lbase != 0 || (int64_t)B.d_l * B.d_r >= (1ll << 31)) return;
    const int h = s->hub.h;
    const uint32_t lomask = (1u << h) - 1u;
    const int32_t nr = B.d_l;
    // up segments: maximal runs of rows with the same high half
    std::vector<int32_t> seg_of_row(nr), seg_row0, seg_rows;
    std::map<uint32_t, int32_t> seg_of_hi;
    for (int32_t a = 0; a < nr; ++a) {
        const uint32_t hi = s->lwords[a] >> h;
        if (a == 0 || hi != (s->lwords[a - 1] >> h)) {
            if (seg_of_hi.count(hi)) return;   // not contiguous
            seg_of_hi[hi] = (int32_t)seg_row0.size();
            seg_row0.push_back(a);
            seg_rows.push_back(0);
        }
        seg_of_row[a] = (int32_t)seg_row0.size() - 1;
        ++seg_rows.back();
    }
    const int32_t ns = (int32_t)seg_row0.size();
    std::vector<std::vector<int32_t>> hnb(ns);
    s->hs_ulo.assign((size_t)nr * 9, 0);
    s->hs_ucross.assign(nr, -1);
    for (int32_t a = 0; a < nr; ++a) {
        const uint32_t w = s->lwords[a];
        const int32_t g = seg_of_row[a], i = a - seg_row0[g];
        std::vector<int32_t> his;
        int nlo = 0;
        for (int32_t q = s->hl_ptr[a]; q < s->hl_ptr[a + 1]; ++q) {
            const int32_t a2 = s->hl_col[q];
            if (a2 == a || a2 < 0 || a2 >= nr) return;
            const uint32_t w2 = s->lwords[a2];
            if ((w2 >> h) == (w >> h)) {
                if (nlo == 8) return;
                s->hs_ulo[(size_t)a * 9 + 1 + nlo++] = a2 - a;
            } else if ((w2 & lomask) == (w & lomask)) {
                const int32_t g2 = seg_of_row[a2];
                if (a2 - seg_row0[g2] != i || seg_rows[g2] != seg_rows[g]) return;
                his.push_back(seg_row0[g2]);
            } else {
                if (s->hs_ucross[a] >= 0) return;
                s->hs_ucross[a] = a2;
            }
        }
        s->hs_ulo[(size_t)a * 9] = nlo;
        std::sort(his.begin(), his.end());
        if (i == 0) hnb[g] = his;
        else if (his != hnb[g]) return;   // the high-half hops must not depend on the low half
    }
    size_t uhs = 1;
    for (auto &v : hnb) uhs = std::max(uhs, v.size());
    for (int32_t g = 0; g < ns; ++g) {
        s->hs_useg.insert(s->hs_useg.end(), {seg_row0[g], seg_rows[g], seg_row0[g], (int32_t)hnb[g].size()});
        for (size_t q = 0; q < uhs; ++q) s->hs_uhnb.push_back(q < hnb[g].size() ? hnb[g][q] : seg_row0[g]);
    }
    s->hs_uhs = (int32_t)uhs;
    // items: panels (up segment x down class), heaviest first, dealt to 8
    // equal XCD chunks padded with empty items
    const int n_cls = (int)(s->hc_cls.size() / 8);
    struct Panel {
        int64_t size;
        int32_t g, ci;
    };
    std::vector<Panel> panels;
    int32_t max_tile = 1;
    for (int32_t g = 0; g < ns; ++g)
        for (int ci = 0; ci < n_cls; ++ci) {
            const int L = s->hc_cls[8 * ci], nseg = s->hc_cls[8 * ci + 1];
            const int per_pass = HUBSEG_THREADS / L;
            if (per_pass < 1 || (seg_rows[g] + per_pass - 1) / per_pass > HUBSEG_M) return;
            max_tile = std::max(max_tile, seg_rows[g] * (L + 1));
            panels.push_back(Panel{(int64_t)seg_rows[g] * L * nseg, g, ci});
        }
    if ((size_t)max_tile * 8 > 48 * 1024) return;
    std::stable_sort(panels.begin(), panels.end(), [](const Panel &x, const Panel &y) { return x.size > y.size; });
    const int n_chunks = 8;
    std::vector<std::vector<HubSegItem>> ch(n_chunks);
    std::vector<int64_t> load(n_chunks, 0);
    int32_t slot = 0;
    for (const Panel &P : panels) {
        // the least loaded chunk takes the next panel
        const int c = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[c] += P.size;
        const int nseg = s->hc_cls[8 * P.ci + 1], seg_base = s->hc_cls[8 * P.ci + 2];
        for (int si = 0; si < nseg; ++si) ch[c].push_back(HubSegItem{P.g, seg_base + si, P.ci, slot++});
    }
    size_t len = 0;
    for (auto &c : ch) len = std::max(len, c.size());
    for (auto &c : ch) {
        s->hs_items.insert(s->hs_items.end(), c.begin(), c.end());
        for (size_t k = c.size(); k < len; ++k) s->hs_items.push_back(HubSegItem{-1, 0, 0, 0});
    }
    s->hs_n_slots = slot;
    s->hs_max_tile = max_tile;
    s->hubseg_ok = true;
}

// Tables of the two-pass flat kernels: the down-spin operator H_dn in column
// space (class-major columns), one slot per bond: col[b * d_R + c] is the
// column reached from column c by a hop across bond b, or -1 if the bond
// cannot hop there (both sites empty or both occupied); val[b * d_R + c] its
// value -t_b times the fermion sign.  Bond-major slots make the gathers of a
// wave for one bond touch neighbouring addresses: a hop inside the high half
// moves a whole segment of columns by the same offset, a hop inside the low
// half stays in the segment.  The values are dropped when every hop of both
// spins has the same value (the kernels then scale the neighbour sums once).
static void build_hub6_tables(ecut_sectors *s, const ecut_model_desc *m) {
    s->hub6_ok = false;
    const BlockDev &B = s->blocks[0];
    const int64_t dR = B.d_r;
    if (dR < 1 || B.d_l < 1 || dR >= (1ll << 30)) return;
    std::vector<int> bonds;
    for (int b = 0; b < m->n_bonds; ++b)
        if (m->t[b] != 0.0) bonds.push_back(b);
    const int nb = (int)bonds.size();
    if (nb > HUBD_MAX_SLOTS || (int64_t)std::max(nb, 1) * dR >= (1ll << 31)) return;
    bool uniform = true;
    double hop = 0.0;
    bool have = false;
    for (const std::vector<double> *v : {&s->hl_val, &s->hr_val})
        for (double x : *v) {
            if (!have) { hop = x; have = true; }
            uniform = uniform && x == hop;
        }
    s->h6_uniform = uniform;
    s->h6_hop = hop;
    s->h6_maxq = nb;
    s->h6_col.assign(std::max<int64_t>(1, (int64_t)nb * dR), -1);
    s->h6_val.clear();
    if (!uniform) s->h6_val.assign(std::max<int64_t>(1, (int64_t)nb * dR), 0.0);
    for (int64_t c = 0; c < dR; ++c) {
        const uint32_t w = s->hub_rw32[c];
        for (int k = 0; k < nb; ++k) {
            const int b = bonds[k];
            uint32_t w2;
            int sg;
            if (!fermion_hop(w, m->bond_i[b], m->bond_j[b], w2, sg) && !fermion_hop(w, m->bond_j[b], m->bond_i[b], w2, sg))
                continue;
            s->h6_col[(size_t)k * dR + c] = s->hub_col_of_rank[colex_rank(w2)];
            if (!uniform) s->h6_val[(size_t)k * dR + c] = -m->t[b] * sg;
        }
    }
    s->hub6_ok = true;
}

// Column of the down word of canonical rank r in the block (identity unless
// the Hubbard up/down kernels, which use the class-major column order, apply).
int32_t hub_column(const ecut_sectors *s, int64_t r) {
    return s->hub_ok ? s->hub_col_of_rank[(size_t)r] : (int32_t)r;
}

static void make_rank_tables(ecut_sectors *s) {
    s->spin_rank_lo.assign(256, 0);
    s->spin_rank_hi.assign(256 * 9, 0);
    for (uint32_t lo = 0; lo < 256; ++lo) {
        int t = 0;
        int64_t r = 0;
        for (int p = 0; p < 8; ++p)
            if ((lo >> p) & 1u) r += (int64_t)binom(p, ++t);
        s->spin_rank_lo[lo] = (int32_t)r;
    }
    for (uint32_t hi = 0; hi < 256; ++hi)
        for (int c = 0; c <= 8; ++c) {
            int t = c;
            int64_t r = 0;
            for (int p = 0; p < 8; ++p)
                if ((hi >> p) & 1u) r += (int64_t)binom(8 + p, ++t);
            s->spin_rank_hi[hi * 9 + c] = (int32_t)r;
        }
}

// Tables of the whole-row Hubbard kernel: every bond with t != 0 as the
// mask of its two sites, the mask of the sites strictly between them (the
// fermion sign of a hop is the parity of the particles there) and -t.
// Needs down words of at most 16 bits (byte-table ranking), an even row
// length (16-byte column pairs) and a row that fits the work group.
static void build_hubrow_tables(ecut_sectors *s, const ecut_model_desc *m) {
    s->hubrow_ok = false;
    const BlockDev &B = s->blocks[0];
    if (s->n_sites > 16 || B.d_r % 2 != 0 || B.d_r > HUBROW_COLS || B.d_r < 2) return;
    s->hrow_bmask.clear();
    s->hrow_bbetw.clear();
    s->hrow_bcoef.clear();
    for (int b = 0; b < m->n_bonds; ++b) {
        if (m->t[b] == 0.0) continue;
        const int i = std::min(m->bond_i[b], m->bond_j[b]), j = std::max(m->bond_i[b], m->bond_j[b]);
        s->hrow_bmask.push_back((1u << i) | (1u << j));
        s->hrow_bbetw.push_back(((1u << j) - 1u) & ~((1u << (i + 1)) - 1u));
        s->hrow_bcoef.push_back(-m->t[b]);
    }
    if (s->hrow_bmask.size() > (size_t)HUBROW_MAX_BOND) return;
    make_rank_tables(s);
    s->hubrow_ok = true;
}

// Tables of the spin kernel.  The colex rank of a word w of up to 16 bits,
// sum over its set bits p_0 < p_1 < ... of C(p_t, t+1), splits into a part
// that depends only on the low byte and a part that depends on the high byte
// and the popcount of the low byte:
//   rank(w) = rank_lo[w & 255] + rank_hi[(w >> 8) * 9 + popc(w & 255)].
// The tables do not depend on the sector, so one pair serves every block.
// The Sz Sz cross terms coef (s_i - 1/2)(s_j - 1/2) (i in L, j in R) of one
// amplitude, grouped by j: sum_j (s_j - 1/2) G_j(l) with
// G_j(l) = sum over the terms on j of coef (s_i(l) - 1/2), in term order.
// The table holds G_j / 2 per left word, so a kernel adds +-G_j/2 per right
// site (exact: s_j - 1/2 is +-1/2).  At most XR_MAX distinct right sites.
static void fold_cross_diagonal(ecut_sectors *s) {
    s->xdl.clear();
    s->xr_site.clear();
    if (s->kind != ECUT_SPIN_HALF || s->xdiag.empty()) return;
    std::vector<int32_t> sites;
    for (const XDiagDev &X : s->xdiag)
        if (std::find(sites.begin(), sites.end(), X.rj) == sites.end()) sites.push_back(X.rj);
    if (sites.size() > (size_t)XR_MAX) return;
    std::sort(sites.begin(), sites.end());
    const size_t nl = s->lwords.size(), nr = sites.size();
    s->xdl.assign(nl * nr, 0.0);
    for (size_t g = 0; g < nl; ++g) {
        const uint32_t lw = s->lwords[g];
        for (size_t k = 0; k < nr; ++k) {
            double G = 0.0;
            for (const XDiagDev &X : s->xdiag)
                if (X.rj == sites[k]) G += X.coef * ((double)((lw >> X.li) & 1u) - 0.5);
            s->xdl[g * nr + k] = 0.5 * G;
        }
    }
    s->xr_site = sites;
}

static void build_spin_tables(ecut_sectors *s) {
    s->spin_ok = false;
    if (s->kind != ECUT_SPIN_HALF) return;
    if (s->lsites.size() > 16 || s->rsites.size() > 16) return;
    if (s->spin_fmask.size() > (size_t)SPIN_MAX_FLIP) return;
    if (s->max_d_r > SPIN_TILE) return;
    s->item_slots = make_spin_items(s, SPIN_MANY_TILE, 0, s->items);
    // every item holds at least one row, so no tile size gives more slots
    // than there are rows; an XCD-dealt list pads each of its 8 chunks to the
    // longest, at most 8 times the items
    size_t rows = 0;
    for (const BlockDev &B : s->blocks) rows += (size_t)B.d_l;
    s->item_slots_cap = (int32_t)std::max(s->items.size(), rows);
    s->items_cap = 8 * (size_t)s->item_slots_cap;
    make_rank_tables(s);
    build_two_pass_tables(s, (int)s->lsites.size(), {});
    s->spin_ok = true;
}

// Tables of the two-pass row kernels (spin problems and the spatial Hubbard
// cut), for left words of lbits bits:
//  - the rows of every block by inversion level of the left word (a hop or
//    flip-flop on bond (i, j) moves a word at most |i - j| levels, so the
//    neighbour rows of a level lie in the levels next to it), and the left
//    operator's CSR in that order;
//  - per block, the source column of every right term (spin_fmask /
//    spin_fcoef: a flip-flop or a hop of one spin, with the fermion sign
//    (-1)^popc(w & rbetw[f]) when rbetw is given) and of every cross term
//    (the right word with bit rj flipped; on the spatial Hubbard cut with
//    the right part's sign (-1)^(occupied modes before the mode)), in the
//    low 15 bits, the sign in bit 15, 0xffff for no term. On a spin cut
//    (no signs) a flip entry is the column's byte offset in the staged row,
//    8 * column, and "no term" is 8 * d_r, the zero slot after the row; a
//    cross entry is the source block's zero slot minus the column, in bytes.
static void build_two_pass_tables(ecut_sectors *s, int lbits, const std::vector<uint32_t> &rbetw) {
    s->sp2_ok = false;
    if (s->spin_fmask.size() > (size_t)SPIN_MAX_FLIP || s->max_d_r > SPIN_TILE) return;
    const int nR = (int)s->rsites.size();
    const bool fermion = s->hub_spatial;
    // a right word's column inside its group
    auto rank = [&](uint32_t w) -> int64_t {
        if (!fermion) return colex_rank(w);
        const uint32_t dn = w & ((1u << nR) - 1u), up = w >> nR;
        return colex_rank(up) * (int64_t)binom(nR, __builtin_popcount(dn)) + colex_rank(dn);
    };
    // occupied modes of the right word before mode (spin, site k): up modes
    // first, then down modes, each by site
    auto occ_before = [&](uint32_t w, int spin, int k) {
        const uint32_t dn = w & ((1u << nR) - 1u), up = w >> nR, below = (1u << k) - 1u;
        return spin == 0 ? __builtin_popcount(up & below) : __builtin_popcount(up) + __builtin_popcount(dn & below);
    };
    s->sp_level_rows.assign(s->lwords.size(), 0);
    for (const BlockDev &B : s->blocks) {
        std::vector<int64_t> key((size_t)B.d_l);
        for (int32_t a = 0; a < B.d_l; ++a)
            key[a] = (int64_t)inversions(s->lwords[(size_t)B.lbase + a], lbits) << 32 | a;
        std::sort(key.begin(), key.end());
        for (int32_t a = 0; a < B.d_l; ++a) s->sp_level_rows[(size_t)B.lbase + a] = (int32_t)(key[a] & 0xffffffff);
    }
    const bool csr_ok = processing_csr(s, s->sp_level_rows, s->sp_pptr, s->sp_pcol, s->sp_pval) <= 64;
    const int nf = (int)s->spin_fmask.size(), ng = (nf + 3) / 4, nx = (int)s->xbond.size();
    s->sp_tbase.assign(2 * s->blocks.size(), 0);
    int64_t n = 0;
    for (size_t b = 0; b < s->blocks.size(); ++b) {
        s->sp_tbase[2 * b] = n;
        n += (int64_t)ng * 4 * s->blocks[b].d_r;
        s->sp_tbase[2 * b + 1] = n;
        n += (int64_t)nx * s->blocks[b].d_r;
        n = (n + 3) & ~(int64_t)3;   // 8-byte aligned groups
    }
    s->sp_tab.assign((size_t)std::max<int64_t>(n, 4), 0xffff);
    // "no term" in a flip table: 0xffff with fermion signs; for spin cuts the
    // byte offset of the zero slot the kernel keeps after the row (8 * d_r),
    // so a term that does not apply (and a pad entry) reads 0 with no test
    static_assert(SPIN_TILE * 8 < 0xffff, "a spin cut's byte offsets fit 16 bits");
    const int64_t unit = fermion ? 1 : 8;   // a spin cut's entries are byte offsets
    if (!fermion)
        for (size_t b = 0; b < s->blocks.size(); ++b)
            std::fill(s->sp_tab.begin() + s->sp_tbase[2 * b],
                      s->sp_tab.begin() + s->sp_tbase[2 * b] + (int64_t)ng * 4 * s->blocks[b].d_r,
                      (uint16_t)(8 * s->blocks[b].d_r));
    for (size_t b = 0; b < s->blocks.size(); ++b) {
        const BlockDev &B = s->blocks[b];
        for (int32_t e = 0; e < B.d_r; ++e) {
            const uint32_t w = s->rwords[(size_t)B.rbase + e];
            for (int f = 0; f < nf; ++f)
                if (__builtin_popcount(w & s->spin_fmask[f]) == 1) {
                    const int sg = rbetw.empty() ? 0 : (__builtin_popcount(w & rbetw[f]) & 1);
                    s->sp_tab[(size_t)(s->sp_tbase[2 * b] + ((int64_t)(f / 4) * B.d_r + e) * 4 + f % 4)] =
                        (uint16_t)(unit * rank(w ^ s->spin_fmask[f]) | (sg << 15));
                }
            for (int k = 0; k < nx; ++k) {
                const XBondDev &X = s->xbond[k];
                const uint32_t wp = w ^ (1u << X.rj);
                uint16_t v;
                if (fermion) {
                    const int sg = occ_before(w, X.label, X.label ? X.rj : X.rj - nR) & 1;
                    v = (uint16_t)(rank(wp) | (sg << 15));
                } else {
                    // the source block's zero slot minus the source column, in
                    // bytes: the kernel subtracts it from the zero slot when the
                    // term applies (a source block too wide for the kernel does
                    // not exist in a problem on it, and its entry is never read)
                    const int64_t z = 8 * (int64_t)binom(nR, __builtin_popcount(wp));
                    v = z <= 8 * (int64_t)s->max_d_r ? (uint16_t)(z - 8 * rank(wp)) : (uint16_t)0;
                }
                s->sp_tab[(size_t)(s->sp_tbase[2 * b + 1] + (int64_t)k * B.d_r + e)] = v;
            }
        }
    }
    spin_left_blocks(s, HUBU_ROWS, s->sp_lblocks);
    s->sp2_ok = csr_ok && s->max_d_r < 32768;
}

int32_t processing_csr(const ecut_sectors *s, const std::vector<int32_t> &order, std::vector<int32_t> &pptr,
                       std::vector<int32_t> &pcol, std::vector<double> &pval) {
    const size_t n = s->lwords.size();
    std::vector<int64_t> src(n, -1);   // processing position -> global row
    for (const BlockDev &B : s->blocks)
        for (int32_t p = 0; p < B.d_l; ++p) src[(size_t)B.lbase + p] = (int64_t)B.lbase + order[(size_t)B.lbase + p];
    pptr.assign(n + 1, 0);
    pcol.clear();
    pval.clear();
    int32_t maxd = 0;
    for (size_t p = 0; p < n; ++p) {
        if (src[p] >= 0) {
            const int32_t q0 = s->hl_ptr[(size_t)src[p]], q1 = s->hl_ptr[(size_t)src[p] + 1];
            pcol.insert(pcol.end(), s->hl_col.begin() + q0, s->hl_col.begin() + q1);
            pval.insert(pval.end(), s->hl_val.begin() + q0, s->hl_val.begin() + q1);
            maxd = std::max(maxd, q1 - q0);
        }
        pptr[p + 1] = (int32_t)pcol.size();
    }
    if (pcol.empty()) {   // keep the device arrays non-empty
        pcol.push_back(0);
        pval.push_back(0.0);
    }
    return maxd;
}

// Left-pass block table of the two-pass spin kernels for items of
// `rows_per_item` rows: slabs of 64 columns, every block with amplitudes.
void spin_left_blocks(const ecut_sectors *s, int32_t rows_per_item, std::vector<SpinLBlock> &out) {
    out.clear();
    int32_t item0 = 0;
    for (const BlockDev &B : s->blocks) {
        if ((int64_t)B.d_l * B.d_r == 0) continue;
        SpinLBlock L{};
        L.offset = B.offset;
        L.d_l = B.d_l;
        L.d_r = B.d_r;
        L.lbase = B.lbase;
        L.item0 = item0;
        L.n_rgroups = (B.d_l + rows_per_item - 1) / rows_per_item;
        L.n_slabs = (B.d_r + 63) / 64;
        item0 += L.n_rgroups * L.n_slabs;
        out.push_back(L);
    }
}

// Work items of the spin kernel: a row longer than half the tile is an item of
// its own (its cross-term source rows are staged in LDS), shorter rows are
// packed into items of at most `tile` amplitudes; largest first.
//
// Order 1 deals the items to 8 chunks, one per XCD: the one-row items of a
// block in runs that share the high half of the left word (a segment, whose
// rows are each other's neighbours under the left bonds inside the low half),
// every run to the chunk with the least work so far.  The chunks are padded
// to one length with empty items and interleaved, position 8 k + c holding
// item k of chunk c, so a grid-stride walk with a grid that is a multiple of
// 8 runs chunk c on XCD c (work group w runs on XCD w % 8).
//
// Order 2 (the two-pass kernels) puts the one-row items first, grouped by the
// interior of the left word, then the items of several rows.
int32_t make_spin_items(const ecut_sectors *s, int32_t tile, int32_t order, std::vector<ItemDev> &out) {
    std::vector<ItemDev> base;
    for (int b = 0; b < (int)s->blocks.size(); ++b) {
        const BlockDev &B = s->blocks[b];
        const int32_t rpt = std::max<int32_t>(1, std::min<int32_t>(B.d_l, tile / std::max(B.d_r, 1)));
        for (int32_t r0 = 0; r0 < B.d_l; r0 += rpt) base.push_back(ItemDev{0, b, r0, std::min(B.d_l, r0 + rpt), 0, 0});
    }
    auto work = [&](const ItemDev &a) { return (int64_t)(a.row1 - a.row0) * s->blocks[a.block].d_r; };
    std::stable_sort(base.begin(), base.end(), [&](const ItemDev &a, const ItemDev &b) { return work(a) > work(b); });
    for (size_t k = 0; k < base.size(); ++k) base[k].slot = (int32_t)k;
    const int32_t n_slots = (int32_t)base.size();
    if (order == 2) {
        // one-row items first, grouped by the left sites that no cross term
        // touches: the cross-term source rows of a row differ from it only
        // at the cut's left sites, so the rows of one group (in every block)
        // are each other's source rows
        uint32_t bmask = 0;
        for (const XBondDev &X : s->xbond) bmask |= 1u << X.li;
        auto key = [&](const ItemDev &a) {
            const uint32_t w = s->lwords[(size_t)s->blocks[a.block].lbase + a.row0];
            return (uint64_t)(w & ~bmask) << 32 | (w & bmask);
        };
        std::vector<ItemDev> one, many;
        for (const ItemDev &a : base) (a.row1 - a.row0 == 1 ? one : many).push_back(a);
        std::stable_sort(one.begin(), one.end(), [&](const ItemDev &a, const ItemDev &b) { return key(a) < key(b); });
        out = one;
        out.insert(out.end(), many.begin(), many.end());
        return n_slots;
    }
    if (order != 1) {
        out.swap(base);
        return n_slots;
    }
    const int n_chunks = 8;
    const int hshift = ((int)s->lsites.size() + 1) / 2;
    std::vector<std::vector<ItemDev>> ch(n_chunks);
    std::vector<int64_t> load(n_chunks, 0);
    size_t k = 0;
    while (k < base.size()) {
        const ItemDev &a = base[k];
        size_t k1 = k + 1;
        if (a.row1 - a.row0 == 1) {
            const BlockDev &B = s->blocks[a.block];
            const uint32_t seg = s->lwords[B.lbase + a.row0] >> hshift;
            while (k1 < base.size() && base[k1].block == a.block && base[k1].row1 - base[k1].row0 == 1 &&
                   (s->lwords[B.lbase + base[k1].row0] >> hshift) == seg)
                ++k1;
        }
        const int c = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t q = k; q < k1; ++q) {
            ch[c].push_back(base[q]);
            load[c] += work(base[q]);
        }
        k = k1;
    }
    size_t len = 0;
    for (auto &c : ch) len = std::max(len, c.size());
    out.assign(len * n_chunks, ItemDev{0, 0, 0, 0, -1, 0});
    for (int c = 0; c < n_chunks; ++c)
        for (size_t i = 0; i < ch[c].size(); ++i) out[i * n_chunks + c] = ch[c][i];
    return n_slots;
}

void make_hub_item_order(const ecut_sectors *s, int order, std::vector<HubItem> &out) {
    // order % 3 picks the row order; 0..2 class major, 3..5 the classes of one
    // row together, 6..8 class major with up-segments (rows sharing the high
    // half of the up word) dealt round-robin to 8 equal chunks, one per XCD,
    // padded with empty items, so each XCD holds whole segments while all
    // XCDs walk the same part of the row order.  9 and 10 take row order 3
    // (up class, then inversion level), class major and row major.
    std::vector<int32_t> ro;
    make_row_order(s, row_order_kind(order), ro);
    std::vector<int32_t> pos(ro.size());
    for (size_t k = 0; k < ro.size(); ++k) pos[ro[k]] = (int32_t)k;
    out = s->hub_items;
    const bool class_major = order < 3 || (order >= 6 && order != 10);
    std::stable_sort(out.begin(), out.end(), [&](const HubItem &a, const HubItem &b) {
        const int64_t ka = class_major ? ((int64_t)a.cls << 32 | pos[a.row0]) : ((int64_t)pos[a.row0] << 8 | a.cls);
        const int64_t kb = class_major ? ((int64_t)b.cls << 32 | pos[b.row0]) : ((int64_t)pos[b.row0] << 8 | b.cls);
        return ka < kb;
    });
    if (order < 6 || order >= 9) return;
    const int n_chunks = 8;
    const int hshift = s->n_sites / 2;
    std::vector<std::vector<HubItem>> ch(n_chunks);
    int g = -1;
    int64_t last_key = -1;
    for (const HubItem &it : out) {
        const uint32_t w = s->lwords[s->blocks[0].lbase + it.row0];
        const int64_t key = ((int64_t)it.cls << 32) | (w >> hshift);
        if (key != last_key) { ++g; last_key = key; }
        ch[g % n_chunks].push_back(it);
    }
    size_t len = 0;
    for (auto &c : ch) len = std::max(len, c.size());
    out.clear();
    for (auto &c : ch) {
        out.insert(out.end(), c.begin(), c.end());
        for (size_t k = c.size(); k < len; ++k) out.push_back(HubItem{0, 0, 0, -1});
    }
}

// Inversion number of an occupation word: pairs (particle at p, hole at q > p).
// A hop of one particle to a neighbouring site changes it by exactly one.
static int inversions(uint32_t w, int n) {
    int inv = 0, holes_above = 0;
    for (int p = n - 1; p >= 0; --p) {
        if ((w >> p) & 1u) inv += holes_above;
        else ++holes_above;
    }
    return inv;
}

void make_row_order(const ecut_sectors *s, int order, std::vector<int32_t> &out) {
    const BlockDev &B = s->blocks[0];
    const int n = s->n_sites;
    out.resize(B.d_l);
    for (int32_t a = 0; a < B.d_l; ++a) out[a] = a;
    if (order == 0) return;
    std::vector<int64_t> key(B.d_l);
    const int h = n / 2;
    for (int32_t a = 0; a < B.d_l; ++a) {
        const uint32_t w = s->lwords[B.lbase + a];
        if (order == 1) {
            key[a] = (int64_t)inversions(w, n) << 32 | a;
        } else if (order == 3) {
            // class of the high half, then inversion level: every hop inside a
            // class moves one level, so the source rows of a level lie in the
            // levels next to it
            key[a] = ((int64_t)__builtin_popcount(w >> h) << 56) | ((int64_t)inversions(w, n) << 32) | a;
        } else {
            const uint32_t hi = w >> h;
            key[a] = ((int64_t)__builtin_popcount(hi) << 56) | ((int64_t)inversions(hi, n - h) << 40) |
                     ((int64_t)hi << 24) | (w & ((1u << h) - 1u));
        }
    }
    std::stable_sort(out.begin(), out.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
}

}  // namespace ecut
