/*
 * oracle.c -- plain CPU FP64 reference for the Hamiltonian application and
 * the Lanczos ground-state energy of the models the paper benchmarks.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library.  It shares no code, header,
 * table or helper with the GPU library; the two meet only through the seeded
 * input generators.
 *
 * What it computes (all in the full occupation basis of one symmetry sector,
 * never in the bipartite form the GPU path uses):
 *   - the sector basis: every occupation word with the requested particle
 *     numbers, in increasing integer order (the symmetry sectors of Eq. 1);
 *   - rows of the K-local Hamiltonian of Eq. (1) for two model families:
 *       spin-1/2:  H = sum_b jxy_b (Sx_i Sx_j + Sy_i Sy_j) + jz_b Sz_i Sz_j,
 *                  S = sigma/2, site i = bit i, spin up = bit set;
 *       Hubbard:   H = -sum_b t_b sum_s (c+_{i s} c_{j s} + h.c.)
 *                      + sum_i U_i n_{i up} n_{i dn},
 *                  word = (up_bits << L) | dn_bits, fermion signs taken from
 *                  the ordered product of creation operators, up modes first
 *                  then down modes, each by increasing site;
 *   - y = H x, either through an explicit CSR matrix or row by row;
 *   - the map from the canonical (integer-ordered) basis to the bipartite
 *     block layout of Eq. (3): block q = (q_l, q_r) by ascending q_l,
 *     row = index of the left word in its sorted list, column = index of the
 *     right word in its sorted list (enumeration + binary search, no ranking
 *     formula);
 *   - textbook Lanczos (the Krylov core the paper builds on) with optional
 *     repeated classical Gram-Schmidt, and eigenvalues of the tridiagonal
 *     matrix by Sturm-sequence bisection.
 *
 * Pins: tests/test_oracle_pins.py checks every function against what the
 * paper and the mathematics fix (dense Kronecker-product Hamiltonians on tiny
 * lattices, closed-form energies, brute-force enumeration, Hermiticity, the
 * Vec/Kronecker identity of the cross term, Sturm bisection against LAPACK),
 * and tests/test_oracle_plants.py shows those pins fail for planted mistakes
 * (compile-time ORC_PLANT, never set in the normal build).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_SPIN = 1, ORC_HUBBARD = 2 };
enum { ORC_CUT_SPATIAL = 1, ORC_CUT_UPDN = 2 };

typedef struct {
    int32_t kind;      /* ORC_SPIN or ORC_HUBBARD */
    int32_t n_sites;   /* S */
    int32_t n_bonds;
    int32_t pad_;
    const int32_t *bi, *bj;   /* bond end points, 0 <= bi, bj < S, bi != bj */
    const double *jxy, *jz;   /* spin couplings per bond */
    const double *t;          /* Hubbard hopping per bond */
    const double *u;          /* Hubbard on-site U per site (may be NULL) */
    const double *v;          /* Hubbard density interaction V n_i n_j per bond,
                                 n = n_up + n_dn (may be NULL) */
} orc_model;

#define ORC_MAX_ROW 1024

/* ORC_PLANT selects one deliberate mistake for the test that shows the pins
 * catch it (tests/test_oracle_plants.py builds each variant into a separate
 * library); the normal build leaves it 0.
 *   1: drop the on-site U term        2: drop the fermion sign of hops
 *   3: flip amplitude jxy, not jxy/2  4: Sz Sz with the first site twice
 *   5: only the down spins hop        6: wrong sign of the beta term in Lanczos
 *   7: Lanczos stops after one step within tol instead of three
 *   8: c+ / c of one mode without its fermion sign
 *   9: drop the bond density interaction V
 *  10: spatial Hubbard cut without the reordering sign */
#ifndef ORC_PLANT
#define ORC_PLANT 0
#endif

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int popcount64(uint64_t w)
{
    int c = 0;
    while (w) { c += (int)(w & 1u); w >>= 1; }
    return c;
}

/* Number of n-bit words with k bits set, by Pascal's rule. */
static int64_t choose(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t row[65];
    for (int j = 0; j <= k; ++j) row[j] = (j == 0);
    for (int i = 1; i <= n; ++i)
        for (int j = (i < k ? i : k); j >= 1; --j) row[j] += row[j - 1];
    return row[k];
}

/* Next larger word with the same number of set bits (the classic
 * "snoob" bit trick, HAKMEM item 175).  Pinned against brute force. */
static uint64_t next_same_popcount(uint64_t w)
{
    uint64_t c = w & (~w + 1);
    uint64_t r = w + c;
    return (((r ^ w) >> 2) / c) | r;
}

/* All n-bit words with k set bits, increasing. Returns the count. */
static int64_t words_with_count(int n, int k, uint64_t *out)
{
    if (k < 0 || k > n) return 0;
    int64_t cnt = choose(n, k);
    if (!out) return cnt;
    if (k == 0) { out[0] = 0; return 1; }
    uint64_t w = (k == 64) ? ~0ull : ((1ull << k) - 1);
    for (int64_t i = 0; i < cnt; ++i) { out[i] = w; if (i + 1 < cnt) w = next_same_popcount(w); }
    return cnt;
}

int64_t orc_sector_size(int kind, int n_sites, int n_up, int n_dn)
{
    if (kind == ORC_SPIN) return choose(n_sites, n_up);
    if (kind == ORC_HUBBARD) return choose(n_sites, n_up) * choose(n_sites, n_dn);
    return -1;
}

/* Sector basis in increasing integer order.  Returns the number of words. */
int64_t orc_enumerate(int kind, int n_sites, int n_up, int n_dn, uint64_t *words)
{
    if (kind == ORC_SPIN) {
        if (n_sites > 63) return -1;
        return words_with_count(n_sites, n_up, words);
    }
    if (kind == ORC_HUBBARD) {
        if (n_sites > 31) return -1;
        int64_t nu = choose(n_sites, n_up), nd = choose(n_sites, n_dn);
        if (!words) return nu * nd;
        uint64_t *up = malloc(sizeof(uint64_t) * (size_t)(nu > 0 ? nu : 1));
        uint64_t *dn = malloc(sizeof(uint64_t) * (size_t)(nd > 0 ? nd : 1));
        words_with_count(n_sites, n_up, up);
        words_with_count(n_sites, n_dn, dn);
        int64_t k = 0;
        for (int64_t a = 0; a < nu; ++a)
            for (int64_t b = 0; b < nd; ++b) words[k++] = (up[a] << n_sites) | dn[b];
        free(up); free(dn);
        return k;
    }
    return -1;
}

/* Brute-force enumeration over all 2^n words (n <= 30): the pin for
 * orc_enumerate's spin branch. */
int64_t orc_enumerate_bruteforce(int n_sites, int n_up, uint64_t *words)
{
    if (n_sites > 30) return -1;
    int64_t k = 0;
    for (uint64_t w = 0; w < (1ull << n_sites); ++w)
        if (popcount64(w) == n_up) { if (words) words[k] = w; ++k; }
    return k;
}

/* Index of w in the sorted list, or -1. */
int64_t orc_find(const uint64_t *words, int64_t n, uint64_t w)
{
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (words[mid] == w) return mid;
        if (words[mid] < w) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ---- fermionic modes, spin-major order: (site 0,up) ... (site L-1,up),
 *      (site 0,dn) ... (site L-1,dn).  Word bit of a mode: up site s lives
 *      at bit L+s, down site s at bit s. ---- */
static int mode_bit(int L, int mode) { return mode < L ? L + mode : mode - L; }

static int mode_occupied(uint64_t w, int L, int mode) { return (int)((w >> mode_bit(L, mode)) & 1u); }

/* Number of occupied modes that precede `mode` in the creation-operator
 * order: the number of anticommutations needed to bring c or c+ of that
 * mode to the front of the ordered product. */
static int occupied_before(uint64_t w, int L, int mode)
{
    int c = 0;
    for (int m = 0; m < mode; ++m) c += mode_occupied(w, L, m);
    return c;
}

/* Apply c+_a c_b to basis word w.  Returns 0 if the result vanishes, else
 * stores the new word and the sign (+1/-1). */
static int apply_hop(uint64_t w, int L, int a, int b, uint64_t *w_out, int *sign)
{
    if (!mode_occupied(w, L, b)) return 0;
    int s = (occupied_before(w, L, b) & 1) ? -1 : 1;
    uint64_t w1 = w & ~(1ull << mode_bit(L, b));
    if (mode_occupied(w1, L, a)) return 0;
    s *= (occupied_before(w1, L, a) & 1) ? -1 : 1;
#if ORC_PLANT == 2
    s = 1;
#endif
    *w_out = w1 | (1ull << mode_bit(L, a));
    *sign = s;
    return 1;
}

/* Entries of H|w> = sum_k val[k] |w_k>.  For a real symmetric H these are
 * also the entries of row w.  Entries may repeat a word; callers sum them. */
static int model_row(const orc_model *m, uint64_t w, uint64_t *cw, double *cv)
{
    int n = 0;
    double diag = 0.0;
    if (m->kind == ORC_SPIN) {
        for (int b = 0; b < m->n_bonds; ++b) {
            int i = m->bi[b], j = m->bj[b];
            int ni = (int)((w >> i) & 1u), nj = (int)((w >> j) & 1u);
#if ORC_PLANT == 4
            nj = ni;
#endif
            double si = ni ? 0.5 : -0.5, sj = nj ? 0.5 : -0.5;
            diag += m->jz[b] * si * sj;
            /* jxy (SxSx + SySy) = jxy/2 (S+_i S-_j + S-_i S+_j): flips an
             * antiparallel pair with amplitude jxy/2. */
            if (ni != nj && m->jxy[b] != 0.0) {
                if (n >= ORC_MAX_ROW - 1) return -1;
                cw[n] = w ^ ((1ull << i) | (1ull << j));
#if ORC_PLANT == 3
                cv[n] = m->jxy[b];
#else
                cv[n] = 0.5 * m->jxy[b];
#endif
                ++n;
            }
        }
    } else {
        int L = m->n_sites;
        if (m->u && ORC_PLANT != 1)
            for (int s = 0; s < L; ++s)
                if (((w >> (L + s)) & 1u) && ((w >> s) & 1u)) diag += m->u[s];
        if (m->v && ORC_PLANT != 9)
            for (int b = 0; b < m->n_bonds; ++b) {
                const int i = m->bi[b], j = m->bj[b];
                const int ni = (int)((w >> (L + i)) & 1u) + (int)((w >> i) & 1u);
                const int nj = (int)((w >> (L + j)) & 1u) + (int)((w >> j) & 1u);
                diag += m->v[b] * ni * nj;
            }
        for (int b = 0; b < m->n_bonds; ++b) {
            if (m->t[b] == 0.0) continue;
            for (int spin = ORC_PLANT == 5 ? 1 : 0; spin < 2; ++spin) {
                int mi = spin * L + m->bi[b], mj = spin * L + m->bj[b];
                uint64_t w2; int sg;
                if (apply_hop(w, L, mi, mj, &w2, &sg)) {
                    if (n >= ORC_MAX_ROW - 1) return -1;
                    cw[n] = w2; cv[n] = -m->t[b] * sg; ++n;
                }
                if (apply_hop(w, L, mj, mi, &w2, &sg)) {
                    if (n >= ORC_MAX_ROW - 1) return -1;
                    cw[n] = w2; cv[n] = -m->t[b] * sg; ++n;
                }
            }
        }
    }
    cw[n] = w; cv[n] = diag; ++n;
    return n;
}

static int model_ok(const orc_model *m)
{
    if (!m || m->n_sites <= 0 || m->n_bonds < 0) return 0;
    if (m->kind == ORC_SPIN && (m->n_sites > 63 || !m->jxy || !m->jz)) return 0;
    if (m->kind == ORC_HUBBARD && (m->n_sites > 31 || !m->t)) return 0;
    if (m->kind != ORC_SPIN && m->kind != ORC_HUBBARD) return 0;
    for (int b = 0; b < m->n_bonds; ++b) {
        if (m->bi[b] < 0 || m->bj[b] < 0 || m->bi[b] >= m->n_sites || m->bj[b] >= m->n_sites) return 0;
        if (m->bi[b] == m->bj[b]) return 0;
    }
    return 1;
}

/* Row r of H (basis word words[r]) as sorted, merged (col, val) pairs. */
static int csr_row(const orc_model *m, const uint64_t *words, int64_t n, int64_t r,
                   int64_t *cols, double *vals)
{
    uint64_t cw[ORC_MAX_ROW]; double cv[ORC_MAX_ROW];
    int k = model_row(m, words[r], cw, cv);
    if (k < 0) return -1;
    int c = 0;
    for (int e = 0; e < k; ++e) {
        int64_t col = orc_find(words, n, cw[e]);
        if (col < 0) return -2;   /* H left the sector: a model error */
        /* insertion into a sorted list, merging equal columns */
        int p = 0;
        while (p < c && cols[p] < col) ++p;
        if (p < c && cols[p] == col) { vals[p] += cv[e]; continue; }
        for (int q = c; q > p; --q) { cols[q] = cols[q - 1]; vals[q] = vals[q - 1]; }
        cols[p] = col; vals[p] = cv[e]; ++c;
    }
    return c;
}

/* Two-pass CSR build.  Pass 1 (col == NULL): fills row_ptr and returns nnz.
 * Pass 2: fills col/val.  Returns nnz or a negative error. */
int64_t orc_build_csr(const orc_model *m, const uint64_t *words, int64_t n,
                      int64_t *row_ptr, int32_t *col, double *val)
{
    if (!model_ok(m)) return -1;
    int err = 0;
    if (!col) {
        row_ptr[0] = 0;
        #pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t r = 0; r < n; ++r) {
            int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
            int c = csr_row(m, words, n, r, cols, vals);
            if (c < 0) { err = c; c = 0; }
            row_ptr[r + 1] = c;
        }
        if (err) return err;
        for (int64_t r = 0; r < n; ++r) row_ptr[r + 1] += row_ptr[r];
        return row_ptr[n];
    }
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < n; ++r) {
        int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
        int c = csr_row(m, words, n, r, cols, vals);
        if (c < 0) { err = c; continue; }
        for (int e = 0; e < c; ++e) { col[row_ptr[r] + e] = (int32_t)cols[e]; val[row_ptr[r] + e] = vals[e]; }
    }
    return err ? err : row_ptr[n];
}

/* CSR of rows [r0, r1) only (columns are still indices into the whole
 * sector): the same two passes as orc_build_csr, row_ptr has r1 - r0 + 1
 * entries starting at 0.  Lets the host baseline time a CSR product on a
 * bounded sample of a sector whose full CSR would not fit in memory. */
int64_t orc_build_csr_rows(const orc_model *m, const uint64_t *words, int64_t n, int64_t r0, int64_t r1,
                           int64_t *row_ptr, int32_t *col, double *val)
{
    if (!model_ok(m) || r0 < 0 || r1 > n || r1 < r0) return -1;
    const int64_t nr = r1 - r0;
    int err = 0;
    if (!col) {
        row_ptr[0] = 0;
        #pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t k = 0; k < nr; ++k) {
            int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
            int c = csr_row(m, words, n, r0 + k, cols, vals);
            if (c < 0) { err = c; c = 0; }
            row_ptr[k + 1] = c;
        }
        if (err) return err;
        for (int64_t k = 0; k < nr; ++k) row_ptr[k + 1] += row_ptr[k];
        return row_ptr[nr];
    }
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t k = 0; k < nr; ++k) {
        int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
        int c = csr_row(m, words, n, r0 + k, cols, vals);
        if (c < 0) { err = c; continue; }
        for (int e = 0; e < c; ++e) { col[row_ptr[k] + e] = (int32_t)cols[e]; val[row_ptr[k] + e] = vals[e]; }
    }
    return err ? err : row_ptr[nr];
}

/* Threads of the OpenMP loops from now on (the host baseline's single-thread
 * and all-core legs). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

void orc_spmv_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                  const double *x, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) acc += val[e] * x[col[e]];
        y[r] = acc;
    }
}

/* y[k] = (H x)[rows[k]] without a stored matrix. */
int orc_apply_rows(const orc_model *m, const uint64_t *words, int64_t n, const double *x,
                   const int64_t *rows, int64_t nrows, double *y)
{
    if (!model_ok(m)) return -1;
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
        int c = csr_row(m, words, n, rows[k], cols, vals);
        if (c < 0) { err = c; continue; }
        double acc = 0.0;
        for (int e = 0; e < c; ++e) acc += vals[e] * x[cols[e]];
        y[k] = acc;
    }
    return err;
}

/* y = H x over the whole sector without a stored matrix. */
int orc_apply_full(const orc_model *m, const uint64_t *words, int64_t n, const double *x, double *y)
{
    if (!model_ok(m)) return -1;
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < n; ++r) {
        int64_t cols[ORC_MAX_ROW]; double vals[ORC_MAX_ROW];
        int c = csr_row(m, words, n, r, cols, vals);
        if (c < 0) { err = c; continue; }
        double acc = 0.0;
        for (int e = 0; e < c; ++e) acc += vals[e] * x[cols[e]];
        y[r] = acc;
    }
    return err;
}

/* y = c+_{site,spin} x (dagger = 1) or c_{site,spin} x (dagger = 0) between
 * two Hubbard sectors: source words ws[ns], destination words wd[nd] (each in
 * increasing integer order).  The mode is (site, up) for spin 0, (site, dn)
 * for spin 1; the sign is (-1)^(occupied modes before it in the creation-
 * operator order), as for the hops of model_row.  y is overwritten. */
int orc_apply_cdag(int n_sites, const uint64_t *ws, int64_t ns, const uint64_t *wd, int64_t nd,
                   int site, int spin, int dagger, const double *x, double *y)
{
    if (site < 0 || site >= n_sites || spin < 0 || spin > 1 || n_sites > 31) return -1;
    const int L = n_sites, mode = spin * L + site;
    for (int64_t k = 0; k < nd; ++k) y[k] = 0.0;
    int err = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ns; ++k) {
        const uint64_t w = ws[k];
        const int occ = mode_occupied(w, L, mode);
        if (occ == (dagger ? 1 : 0)) continue;   /* c+ on an occupied mode, c on an empty one: 0 */
        const int sg = (ORC_PLANT != 8 && (occupied_before(w, L, mode) & 1)) ? -1 : 1;
        const uint64_t w2 = w ^ (1ull << mode_bit(L, mode));
        const int64_t t = orc_find(wd, nd, w2);
        if (t < 0) { err = 1; continue; }
        y[t] = sg * x[k];   /* the map is one-to-one: no two sources share a target */
    }
    return err ? -2 : 0;
}

/* Gather the bits of w found at the set positions of mask into the low bits,
 * in increasing site order. */
static uint64_t compact_bits(uint64_t w, uint64_t mask)
{
    uint64_t out = 0; int k = 0;
    for (int s = 0; s < 64; ++s)
        if ((mask >> s) & 1u) { out |= ((w >> s) & 1u) << k; ++k; }
    return out;
}

/*
 * Canonical -> bipartite positions (Eq. 3).  blocks receives, per block,
 * (q_l, d_L, d_R, offset) with blocks ordered by ascending q_l.  Returns the
 * number of blocks, or a negative error.
 *   spin + spatial cut: left = sites in left_mask, right = the others;
 *   Hubbard + up/down cut: left = up-spin occupation, right = down-spin.
 */
int orc_bipartite_positions(int kind, int cut, int n_sites, uint64_t left_mask, int n_up, int n_dn,
                            const uint64_t *words, int64_t n, int64_t *pos, int64_t *blocks, int max_blocks)
{
    if (kind == ORC_SPIN && cut == ORC_CUT_SPATIAL) {
        uint64_t full = (n_sites == 64) ? ~0ull : ((1ull << n_sites) - 1);
        if (left_mask & ~full) return -1;
        uint64_t right_mask = full & ~left_mask;
        int nL = popcount64(left_mask), nR = n_sites - nL;
        int qmin = n_up - nR > 0 ? n_up - nR : 0, qmax = n_up < nL ? n_up : nL;
        int nb = qmax - qmin + 1;
        if (nb <= 0 || nb > max_blocks) return -2;
        uint64_t *lw[65], *rw[65]; int64_t dl[65], dr[65], off[65];
        int64_t acc = 0;
        for (int q = qmin; q <= qmax; ++q) {
            int b = q - qmin;
            dl[b] = choose(nL, q); dr[b] = choose(nR, n_up - q);
            lw[b] = malloc(sizeof(uint64_t) * (size_t)dl[b]);
            rw[b] = malloc(sizeof(uint64_t) * (size_t)dr[b]);
            words_with_count(nL, q, lw[b]);
            words_with_count(nR, n_up - q, rw[b]);
            off[b] = acc; acc += dl[b] * dr[b];
            blocks[4 * b + 0] = q; blocks[4 * b + 1] = dl[b]; blocks[4 * b + 2] = dr[b]; blocks[4 * b + 3] = off[b];
        }
        int err = 0;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            uint64_t l = compact_bits(words[i], left_mask), r = compact_bits(words[i], right_mask);
            int b = popcount64(l) - qmin;
            if (b < 0 || b >= nb) { err = 1; continue; }
            int64_t li = orc_find(lw[b], dl[b], l), ri = orc_find(rw[b], dr[b], r);
            if (li < 0 || ri < 0) { err = 1; continue; }
            pos[i] = off[b] + li * dr[b] + ri;
        }
        for (int b = 0; b < nb; ++b) { free(lw[b]); free(rw[b]); }
        return err ? -3 : nb;
    }
    if (kind == ORC_HUBBARD && cut == ORC_CUT_SPATIAL)
        return -5;   /* signed map: orc_bipartite_hubbard_spatial */
    if (kind == ORC_HUBBARD && cut == ORC_CUT_UPDN) {
        if (max_blocks < 1) return -2;
        int64_t nu = choose(n_sites, n_up), nd = choose(n_sites, n_dn);
        uint64_t *uw = malloc(sizeof(uint64_t) * (size_t)nu), *dw = malloc(sizeof(uint64_t) * (size_t)nd);
        words_with_count(n_sites, n_up, uw);
        words_with_count(n_sites, n_dn, dw);
        uint64_t dmask = (1ull << n_sites) - 1;
        int err = 0;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = orc_find(uw, nu, words[i] >> n_sites), b = orc_find(dw, nd, words[i] & dmask);
            if (a < 0 || b < 0) { err = 1; continue; }
            pos[i] = a * nd + b;
        }
        free(uw); free(dw);
        blocks[0] = n_up; blocks[1] = nu; blocks[2] = nd; blocks[3] = 0;
        return err ? -3 : 1;
    }
    return -4;
}

/*
 * Hubbard model with a spatial cut: L = the sites of left_mask, R = the
 * others.  The bipartite basis state |l, r> is the ordered product of the
 * creation operators of the occupied L modes (up modes by site, then down
 * modes by site) followed by those of the R modes in the same order, acting
 * on the vacuum; the canonical state of word w orders all up modes by site,
 * then all down modes.  So |w> = sign(w) |l, r>, sign(w) = the parity of the
 * permutation that sorts w's occupied modes from the one order to the other
 * (counted here pair by pair).  Blocks are (N_up_L, N_dn_L) in lexicographic
 * order; a block's rows are its L words (up bits of the L sites, then down
 * bits, each compacted in site order: l = (up_L << n_L) | dn_L) in increasing
 * integer order, its columns likewise its R words.
 * pos[i], sign[i] for the canonical index i; blocks receive rows
 * (N_up_L, N_dn_L, d_L, d_R, offset).  Returns the number of blocks.
 */
int orc_bipartite_hubbard_spatial(int n_sites, uint64_t left_mask, int n_up, int n_dn, const uint64_t *words, int64_t n,
                                  int64_t *pos, int8_t *sign, int64_t *blocks, int max_blocks)
{
    const int S = n_sites;
    if (S > 31) return -1;
    const uint64_t full = (1ull << S) - 1;
    if (left_mask & ~full) return -1;
    const uint64_t rmask = full & ~left_mask;
    const int nL = popcount64(left_mask), nR = S - nL;
    /* subsystem words by (a, b): all 2n-bit words (up << n) | dn with a up and b down bits */
    int nb = 0;
    int64_t off = 0;
    int64_t dl[65 * 33], dr[65 * 33], boff[65 * 33];
    int bidx[33][33];
    for (int a = 0; a <= nL; ++a)
        for (int b = 0; b <= nL; ++b) {
            bidx[a][b] = -1;
            const int ar = n_up - a, br = n_dn - b;
            if (ar < 0 || br < 0 || ar > nR || br > nR) continue;
            if (nb >= max_blocks) return -2;
            dl[nb] = choose(nL, a) * choose(nL, b);
            dr[nb] = choose(nR, ar) * choose(nR, br);
            boff[nb] = off;
            blocks[5 * nb + 0] = a; blocks[5 * nb + 1] = b; blocks[5 * nb + 2] = dl[nb];
            blocks[5 * nb + 3] = dr[nb]; blocks[5 * nb + 4] = off;
            off += dl[nb] * dr[nb];
            bidx[a][b] = nb++;
        }
    int err = 0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t w = words[i];
        const uint64_t up = w >> S, dn = w & full;
        const uint64_t ul = compact_bits(up, left_mask), dl_ = compact_bits(dn, left_mask);
        const uint64_t ur = compact_bits(up, rmask), dr_ = compact_bits(dn, rmask);
        const int a = popcount64(ul), b = popcount64(dl_);
        const int q = bidx[a][b];
        if (q < 0) { err = 1; continue; }
        /* row: rank of (ul << nL) | dl_ among words with a up and b down
         * bits: the up part's position among the a-words times the number
         * of b-words, plus the down part's position (up-major integer order) */
        int64_t ra = 0, rb = 0, rc = 0, rd = 0;
        /* positions by counting the smaller words of the same popcount */
        for (uint64_t x = 0; x < ul; ++x) ra += popcount64(x) == a;
        for (uint64_t x = 0; x < dl_; ++x) rb += popcount64(x) == b;
        for (uint64_t x = 0; x < ur; ++x) rc += popcount64(x) == n_up - a;
        for (uint64_t x = 0; x < dr_; ++x) rd += popcount64(x) == n_dn - b;
        const int64_t row = ra * choose(nL, b) + rb, col = rc * choose(nR, n_dn - b) + rd;
        pos[i] = boff[q] + row * dr[q] + col;
        /* parity: list the occupied modes with their place in either order */
        int gpos[64], bpos[64], k = 0;
        for (int s = 0; s < S; ++s)
            if ((up >> s) & 1u) {
                const int inL = (int)((left_mask >> s) & 1u);
                gpos[k] = s;
                bpos[k] = inL ? s : 2 * S + s;            /* L up, then (later) R up */
                ++k;
            }
        for (int s = 0; s < S; ++s)
            if ((dn >> s) & 1u) {
                const int inL = (int)((left_mask >> s) & 1u);
                gpos[k] = S + s;
                bpos[k] = inL ? S + s : 3 * S + s;        /* L down before R up */
                ++k;
            }
        int inv = 0;
        for (int x = 0; x < k; ++x)
            for (int y = x + 1; y < k; ++y)
                if ((gpos[x] < gpos[y]) != (bpos[x] < bpos[y])) ++inv;
        if (sign) sign[i] = (ORC_PLANT == 10 || !(inv & 1)) ? 1 : -1;
    }
    return err ? -3 : nb;
}

/* ---------------- Lanczos ---------------- */

/* Every `every` steps (0 = never) orc_lanczos prints the step and the lowest
 * Ritz value to stderr: progress of long runs (the stored energies of the
 * largest sectors take minutes). */
static int g_progress_every = 0;

void orc_set_progress(int every) { g_progress_every = every > 0 ? every : 0; }

/* Neumaier-compensated dot product, serial so the result does not depend on
 * the thread count. */
static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double p = a[i] * b[i], t = s + p;
        if (fabs(s) >= fabs(p)) c += (s - t) + p; else c += (p - t) + s;
        s = t;
    }
    return s + c;
}

/* Number of eigenvalues of the symmetric tridiagonal T (diagonal a[0..m-1],
 * off-diagonal b[0..m-2]) that are smaller than x: the count of negative
 * pivots of the LDL^T factorisation of T - x I (Sturm sequence). */
static int sturm_count(const double *a, const double *b, int m, double x)
{
    int neg = 0;
    double d = 1.0;
    for (int k = 0; k < m; ++k) {
        double bb = k > 0 ? b[k - 1] * b[k - 1] : 0.0;
        d = (a[k] - x) - (k > 0 ? bb / d : 0.0);
        if (d == 0.0) d = -1e-300;   /* x hit an eigenvalue of a leading block */
        if (d < 0.0) ++neg;
    }
    return neg;
}

/* k-th smallest eigenvalue (k = 0, 1, ...) of T by bisection, iterated until
 * the bracket stops shrinking. */
double orc_tridiag_eig(const double *a, const double *b, int m, int k)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {   /* Gershgorin discs */
        double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        if (a[i] - r < lo) lo = a[i] - r;
        if (a[i] + r > hi) hi = a[i] + r;
    }
    lo -= 1e-12 * (fabs(lo) + 1.0); hi += 1e-12 * (fabs(hi) + 1.0);
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, m, mid) > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

/*
 * Textbook Lanczos in Paige's ordering, y = H x supplied either by CSR
 * (row_ptr != NULL) or row by row from the model.
 *   v_1 = v0/|v0|;  u = H v_j - beta_{j-1} v_{j-1};  alpha_j = <v_j,u>;
 *   w = u - alpha_j v_j;  [reorth: w -= V (V^T w), done twice];
 *   beta_j = |w|;  v_{j+1} = w / beta_j.
 * Stops after max_steps, at breakdown (beta_j <= 1e-14 |alpha_j|), or once
 * the lowest Ritz value has changed by at most tol for three steps in a row
 * (tol <= 0 disables that test).  energies[j] receives the lowest Ritz value
 * after step j.  basis (n x max_steps doubles) is needed only with reorth.
 * Returns the number of steps taken, or a negative error.
 */
int orc_lanczos(const orc_model *m, const uint64_t *words, int64_t n,
                const int64_t *row_ptr, const int32_t *col, const double *val,
                const double *v0, int max_steps, int reorth, double tol,
                double *alpha, double *beta, double *energies, double *basis)
{
    if (reorth && !basis) return -1;
    double *v = malloc(sizeof(double) * (size_t)n), *vp = calloc((size_t)n, sizeof(double));
    double *u = malloc(sizeof(double) * (size_t)n);
    double *coef = malloc(sizeof(double) * (size_t)(max_steps + 1));
    if (!v || !vp || !u || !coef) { free(v); free(vp); free(u); free(coef); return -2; }
    double nrm = sqrt(dot(v0, v0, n));
    for (int64_t i = 0; i < n; ++i) v[i] = v0[i] / nrm;
    double beta_prev = 0.0;
    int steps = 0, stable = 0;
    for (int j = 0; j < max_steps; ++j) {
        if (reorth) memcpy(basis + (size_t)j * (size_t)n, v, sizeof(double) * (size_t)n);
        int err = 0;
        if (row_ptr) orc_spmv_csr(n, row_ptr, col, val, v, u);
        else err = orc_apply_full(m, words, n, v, u);
        if (err) { steps = -3; break; }
        for (int64_t i = 0; i < n; ++i) u[i] -= (ORC_PLANT == 6 ? -beta_prev : beta_prev) * vp[i];
        double a = dot(v, u, n);
        for (int64_t i = 0; i < n; ++i) u[i] -= a * v[i];
        if (reorth) {
            for (int pass = 0; pass < 2; ++pass) {
                for (int k = 0; k <= j; ++k) coef[k] = dot(basis + (size_t)k * (size_t)n, u, n);
                for (int k = 0; k <= j; ++k) {
                    const double *q = basis + (size_t)k * (size_t)n;
                    for (int64_t i = 0; i < n; ++i) u[i] -= coef[k] * q[i];
                }
            }
        }
        double b = sqrt(dot(u, u, n));
        alpha[j] = a; beta[j] = b;
        steps = j + 1;
        energies[j] = orc_tridiag_eig(alpha, beta, steps, 0);
        if (g_progress_every && (j + 1) % g_progress_every == 0) {
            fprintf(stderr, "[oracle lanczos] step %d E %.15f\n", j + 1, energies[j]);
            fflush(stderr);
        }
        if (j > 0 && tol > 0.0 && fabs(energies[j] - energies[j - 1]) <= tol) {
            if (++stable >= (ORC_PLANT == 7 ? 1 : 3)) break;
        } else stable = 0;
        if (b <= 1e-14 * fabs(a)) break;
        double *tmp = vp; vp = v; v = tmp;
        for (int64_t i = 0; i < n; ++i) v[i] = u[i] / b;
        beta_prev = b;
    }
    free(v); free(vp); free(u); free(coef);
    return steps;
}
