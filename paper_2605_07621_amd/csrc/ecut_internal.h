// Internal structures of libecut: host-side sector description and the
// device-side descriptors the HIP kernels read.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ecut.h"

namespace ecut {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
ecut_status fail(ecut_status st, const std::string &msg);

// ---------------------------------------------------------------- ranking
// Colex (= increasing integer order) ranking of words with a fixed number of
// set bits: rank(w) = sum_j C(p_j, j+1) over set-bit positions p_0 < p_1 < ...
// (combinatorial number system).
uint64_t binom(int n, int k);
int64_t colex_rank(uint64_t w);
uint64_t colex_unrank(int64_t idx, int k);

// ---------------------------------------------------------------- device descriptors
// Everything the H*psi kernels need for one problem lives in one device
// allocation; ProblemDev holds the pointers into it.  Plain old data so it
// can sit in device memory for batched launches.

struct BlockDev {
    int64_t offset;      // first element of the block in the vector
    int32_t d_l, d_r;    // block shape, row-major [l][r]
    int32_t q_l, q_r;    // subsystem particle numbers (spatial Hubbard cut: up-spin numbers)
    int32_t lbase, rbase;        // first word of count q_l (q_r) in the concatenated L (R) tables
    int32_t blk_lminus, blk_lplus;   // block with q_l-1 (q_l+1), or -1
    int32_t q_l2, q_r2;          // spatial Hubbard cut: down-spin numbers of L and R (else 0)
    int32_t blk_l2minus, blk_l2plus; // block with q_l2-1 (q_l2+1) and the same q_l, or -1
};

// Right sites of a spin cut's diagonal cross terms that the row kernels
// fold per left word (more distinct sites: the terms are summed one by one).
constexpr int XR_MAX = 8;

// Diagonal cross term coef * f(l) * f(r); f(l) = n_li (+ n_li2 when
// li2 >= 0, the two spins of a site: its density), and likewise for r;
// spin_form: f = n - 1/2 instead (spin Sz Sz).
struct XDiagDev {
    int32_t li, rj;
    int32_t spin_form;   // 1: s*s (spin Sz Sz), 0: n*n (Hubbard U n_up n_dn, or V n_i n_j with li2/rj2)
    int32_t li2, rj2;    // second occupation bit of the left / right factor, or -1
    int32_t pad;
    double coef;
};

// Sector-changing cross term for one cut bond (i in L, j in R), both
// directions:  coef (S+_i S-_j + S-_i S+_j).
//   dir A (target l has bit i, r lacks bit j): source block q_l-1,
//         l' = lmap_del[l], r' = rmap_ins[r]
//   dir B (target l lacks bit i, r has bit j): source block q_l+1,
//         l' = lmap_ins[l], r' = rmap_del[r]
// Map arrays are indexed by the global (concatenated) word index and give
// the rank inside the target count, or -1.
//
// Spatial Hubbard cut (fermion = 1): the same two directions for one spin of
// a cut bond, coef (c+_{i s} c_{j s} + h.c.) with coef = -t, maps entries
// (rank << 1) | neg where neg is the fermion sign of that side's operator
// (the product of both sides' signs is the term's sign); label 0 moves the
// up-spin numbers (blk_lminus / blk_lplus), label 1 the down-spin ones
// (blk_l2minus / blk_l2plus).
struct XBondDev {
    int32_t li, rj;
    int32_t lmap_del, lmap_ins;   // offsets into maps[]
    int32_t rmap_del, rmap_ins;
    double coef;
    int32_t label, fermion;
};

// Tables of the Hubbard up/down kernel (row = up word a, column = down word b).
// The down word is split into lo = bits [0,h) and hi = bits [h,n): the column
// index is seg_off[hi] + lo_rank[lo], so a hop inside lo moves the column by a
// lo-only delta, a hop inside hi by a hi-only delta, and only bonds that cross
// the split need both.
struct HubDev {
    int32_t n_r, h;              // down-word bits, split position
    int32_t lo_stride, hi_stride;   // max neighbour entries per lo / hi word
    int32_t n_xb;                // crossing bonds
    int32_t uniform_u;           // 1 if every U_i equals u0
    int32_t uniform_t;           // 1 if every hop value equals hop0 (then coef index is unused)
    int32_t n_coef;
    double u0, hop0;
    const int32_t *lo_cnt;       // [2^h]
    const int32_t *lo_ent;       // [2^h][lo_stride] packed (delta << 9) | (neg << 8) | coef_idx
    const int32_t *lo_rank;      // [2^h]
    const int32_t *hi_cnt;       // [2^(n-h)]
    const int32_t *hi_ent;       // [2^(n-h)][hi_stride]
    const int32_t *seg_off;      // [2^(n-h)] column of (hi, first lo), -1 if the segment is empty
    const int32_t *xb;           // [n_xb][4]: lo bit, hi bit (relative to h), coef_idx, pad
    const double *coef;          // [n_coef] hop values (-t_b)
    const double *u;             // [n_sites] U_i
    const uint16_t *rwords16;    // [d_r] down word of each column (n_r <= 16) or NULL
    const uint32_t *rwords32;    // [d_r] down word of each column
    const int32_t *col_of_rank;  // [d_r] column of the down word of canonical rank r
    // whole-row kernel: down-spin hops by ranking the hopped word
    int32_t n_dbond;             // bonds with t != 0
    int32_t dbond_pad_;
    const uint32_t *dbond_mask;  // [n_dbond] the two sites of the bond
    const uint32_t *dbond_betw;  // [n_dbond] sites strictly between them (fermion sign)
    const double *dbond_coef;    // [n_dbond] -t_b
    const int32_t *rank_lo;      // colex byte tables (see the spin kernel)
    const int32_t *rank_hi;
    // Class tiles.  The down basis splits into classes by the popcount k of
    // the high part; a class is nseg segments (one per high word) of L
    // consecutive columns (one per low word of count N_dn - k).  Hops inside
    // lo or inside hi stay in the class, so one (row, class) tile holds every
    // operand of the right operator except the crossing bonds.
    int32_t n_cls;
    int32_t cls_lo_stride, cls_hi_stride;
    int32_t max_tile;            // largest rows_per_item * L * nseg
    int32_t max_nseg;
    int32_t pad_;
    const int32_t *cls;          // [n_cls][8]: L, nseg, seg_base, lo_base, rows_per_item, L*nseg, 0, 0
    const int32_t *cls_segcol;   // [seg_base + s] flat column of segment s
    const int32_t *cls_hiw;      // [seg_base + s] high word of segment s
    const int32_t *cls_hicnt;    // [seg_base + s] entries in the segment's high-hop list
    const int32_t *cls_hient;    // [(seg_base + s) * cls_hi_stride + q] packed (dseg << 9) | (neg << 8) | coef_idx
    const int32_t *cls_low;      // [lo_base + j] low word of rank j
    const int32_t *cls_locnt;    // [lo_base + j]
    const int32_t *cls_loent;    // [(lo_base + j) * cls_lo_stride + q] packed (dj << 9) | (neg << 8) | coef_idx
};

// Arguments of the fast class-tile kernel (open chains: every hop of either
// spin is -t with a plus sign, U uniform, at most one bond across the lo/hi
// split of the down word and it joins bits h-1 and h).  Tiles are stored
// with a row stride of L+1 doubles whose last element is zero, so inactive
// low-hop entries point at it and every gather is unconditional.
struct Hub3Args {
    const double *x;
    double *y;
    const double *z;
    double *partials;
    double xscale, zcoef, hop, u0;
    const double *dscale;             // nullable: xscale = dscale[0], zcoef = dscale[1]
    const int32_t *hl_ptr, *hl_col;   // up-spin hop rows
    const double *hl_val;
    int32_t n_rows, max_l;            // rows; longest class (its low-hop tables are copied to LDS)
    const uint32_t *lwords;           // up words
    const int32_t *cls;               // [n_cls][8] as HubDev::cls
    const int4 *seginfo;              // [seg]: column, high word, crossing column, crossing bit (2 = none)
    const int4 *loinfo;               // [lo]: low word, crossing low rank, crossing bit (2 = none), 0
    const int32_t *looff;             // [lo][8] low-hop offsets j'-j, or L-j (the zero pad) if unused
    const int32_t *hnb;               // [seg][hs] high-hop neighbour segment index
    const int32_t *hcnt;              // [seg] entries of hnb in use
    const struct HubItem *items;
    int32_t n_items, n_xcd, per_xcd, dR;
    int32_t h, hs, max_tile, max_nseg;
};

// Segment-tile kernel: a tile is (up segment) x (down segment), where a
// segment is the set of words that share the high half.  Up segments are
// contiguous row ranges (rows are in increasing word order), down segments
// contiguous column runs (class-major columns).
struct HubSegArgs {
    const double *x;
    double *y;
    const double *z;
    double *partials;
    double xscale, zcoef, hop, u0;
    const double *dscale;             // nullable: xscale = dscale[0], zcoef = dscale[1]
    const uint32_t *lwords;           // up words
    const int32_t *cls;               // [n_cls][8] as HubDev::cls (down classes)
    const int4 *seginfo;              // down segments, as Hub3Args
    const int4 *loinfo;               // down low words, as Hub3Args
    const int32_t *looff;             // down low-hop offsets, as Hub3Args
    const int32_t *hnb;               // down high-hop neighbours (segment index within the class)
    const int32_t *hcnt;              // down high-hop counts
    const int4 *useg;                 // up segments: first row, rows, up low-table base, high hops
    const int32_t *uhnb;              // [up segment][uhs]: first row of each high-hop neighbour segment
    const int32_t *ulo;               // [up low word][9]: hop count, then row offsets i' - i
    const int32_t *ucross;            // [row]: source row of the crossing-bond hop, -1 if none
    const struct HubSegItem *items;
    int32_t n_items, n_xcd, per_xcd, dR;
    int32_t h, hs, uhs, pad_;
};

// Two-pass Hubbard application on flat work items (variant 6).
// Pass 1 (left operator): y[a, c] = sum_a' H_up[a, a'] x[a', c] over a
// column slab (64 lanes x 1 or 2 columns) and a run of rows of the row order;
// items are slab-major, so the blocks an XCD has in flight cover one slab and
// a window of the row order whose neighbour rows stay in its L2.
struct HubUArgs {
    const double *x;
    double *y;
    const int32_t *hl_ptr, *hl_col;   // left-operator CSR, its rows in processing order (at most 64 entries each)
    const double *hl_val;
    const int32_t *rows;              // processing position -> row of the block
    double hop;                       // every hop value when uniform != 0 (the sum is scaled once)
    int32_t uniform;
    int32_t slab_ways;                // slabs side by side in one item (1, 2 or 4), rows split between them
    int32_t n_rows, dR;
    int32_t rows_per_item, n_rgroups; // rows of the order per item, row runs per slab group
    int32_t n_slabs, n_items;         // slab groups (of slab_ways slabs), items
};

// Pass 2 (right operator, diagonal, epilogue): per element (a, c)
//   y = xscale (y_pass1 + sum_q val_q x[a, col_q] + diag(a, c) x[a, c]) - zcoef z
// with the down-spin hops of column c in bond-major slots (col[b * dR + c]).
// An item is a run of rows x 256 columns; items are row-run-major, so the
// blocks in flight on an XCD cover a few whole rows and the in-row gathers hit
// its L2.  One partial <x, y> per item.
struct HubDArgs {
    const double *x;
    double *y;
    const double *z;
    double *partials;
    double xscale, zcoef;
    const double *dscale;             // nullable: xscale = dscale[0], zcoef = dscale[1]
    const int32_t *col;               // [n_slots][dR] source column of the hop across each bond, -1 if none
    const double *val;                // [n_slots][dR] hop value (NULL: every hop is `hop`)
    double hop;
    const uint32_t *lwords;           // up word of each row
    const uint32_t *rwords;           // down word of each column (column order)
    const double *u;                  // [n_sites] U_i
    double u0;
    int32_t uniform_u, n_rows, dR, rows_per_item;
    int32_t n_chunks, n_items, n_slots, pad_;
};

// c+ / c of one (site, spin) mode between two Hubbard up/down sectors: each
// destination element (a', c') reads its source element, or is 0.
struct CdagArgs {
    const double *x;                  // source vector
    double *y;                        // destination vector
    int64_t dim;                      // destination elements
    int32_t dR_dst, dR_src;
    const uint32_t *dst_lwords;       // up word of each destination row
    const uint32_t *dst_rwords;       // down word of each destination column (column order)
    const int32_t *src_col_of_rank;   // column of the source down word of colex rank r (NULL: r)
    const uint64_t *binom;            // [65][65] binomial table
    int32_t site, spin, dagger, pad_;
};

// Left-operator pass of the two-pass spin kernels over every block of a
// problem: block b owns items item0 .. item0 + n_rgroups * n_slabs - 1,
// slab-major like HubUArgs, its rows in level order at rows + lbase.
struct SpinLBlock {
    int64_t offset;
    int32_t d_l, d_r, lbase, item0;
    int32_t n_rgroups, n_slabs;
};
struct SpinLArgs {
    const double *x;
    double *y;
    const int32_t *hl_ptr, *hl_col;   // left-operator CSR in processing order (per block at lbase), local source rows
    const double *hl_val;
    const int32_t *rows;              // per block at lbase: processing position -> local row (level order)
    const SpinLBlock *blocks;
    int32_t n_blocks, n_items, rows_per_item, pad_;
};

// Layout map of the spatial Hubbard cut (canonical index -> block position
// and fermion sign); blocks are (N_up_L, N_dn_L) over the rectangle
// [la0, la0 + nb_a) x [lb0, lb0 + nb_b), lexicographic.
struct HubSpPerm {
    const BlockDev *blocks;
    const uint64_t *binom;
    int64_t dim, n_dn_words;
    uint32_t lmask, rmask;
    int32_t n_up, n_dn, nL, nR;
    int32_t la0, lb0, nb_b, pad_;
};

// Work item of the segment-tile kernel: up segment, down segment (global
// index), down class; slot = index in the order-independent item list.
// useg < 0 marks padding.
struct HubSegItem {
    int32_t useg, dseg, cls, slot;
};

// Work item of the class-tile kernel: rows [row0, row0 + nrows) of one class;
// slot is the item's index in the order-independent item list.
struct HubItem {
    int32_t row0, nrows, cls, slot;
};

struct ProblemDev {
    int32_t kind;                // ECUT_SPIN_HALF / ECUT_HUBBARD
    int32_t n_blocks;
    int32_t n_xdiag, n_xbond;
    const BlockDev *blocks;
    const uint32_t *lwords, *rwords;
    const int32_t *hl_ptr, *hl_col;
    const double *hl_val;
    const int32_t *hr_ptr, *hr_col;
    const double *hr_val;
    const double *diag_l, *diag_r;
    const XDiagDev *xdiag;
    const XBondDev *xbond;
    const int32_t *maps;
    HubDev hub;
    // spin kernel with ranking tables (spatial cut, both sides <= 16 sites)
    int32_t spin_ok;             // tables below are valid
    int32_t n_rflip;             // flip-flop terms inside the right part
    int32_t max_d_r;             // largest right dimension of any block
    const int32_t *rank_lo;      // colex rank of the low byte: 256 entries
    const int32_t *rank_hi;      // colex rank of the high byte given popc(low byte): 256 x 9
    const uint32_t *rflip_mask;  // the two right-part bits of each flip-flop term
    const double *rflip_coef;    // jxy/2 of each term
    // diagonal cross terms of a spin cut folded per left word: for left word
    // gl and the g-th distinct right site xr_site[g] of the terms,
    // xdl[gl * n_xr + g] = 1/2 sum over the terms on that site of coef (s_li - 1/2),
    // so the terms of (l, r) sum to sum_g (bit xr_site[g] of r ? +1 : -1) xdl[...].
    // n_xr = 0: no table (Hubbard, or more than XR_MAX sites)
    const double *xdl;
    int32_t n_xr;
    int32_t xr_site[XR_MAX];
    int32_t xr_lo, xr_contig;    // xr_contig: the sites are xr_lo, xr_lo + 1, ... (one bit field of r)
    int64_t dim;
    // per launch (filled by the launcher)
    const double *x;             // input vector
    double *y;                   // output vector
    const double *z;             // Lanczos: previous vector (nullable)
    double xscale;               // y = xscale * H x - zcoef * z
    double zcoef;
    const double *dscale;        // nullable: the two factors are read from dscale[0], dscale[1]
    double *partials;            // Lanczos: per-item partial <x, y> (nullable)
};

// Launch parameters of the Hubbard kernel chosen by the autotuner.
struct ApplyTuning {
    int32_t grid;     // work groups (0 = default)
    int32_t n_xcd;    // XCD-contiguous work chunks (0 = 8)
    int32_t order;    // row order: 0 increasing, 1 by inversion level, 2 segment-major by level
    int32_t variant;  // Hubbard kernel: 0 class tiles, 1 whole rows
    int32_t tile;     // spin kernel: amplitudes per item of several short rows (0 = default)
};

// Work item: rows [row0, row1) of block `block` of problem `prob`; `slot`
// is the item's index in its own problem's item list (the partial-sum slot,
// independent of what else shares the launch).
struct ItemDev {
    int32_t prob, block, row0, row1, slot, pad;
};

}  // namespace ecut

// ---------------------------------------------------------------- the handle
struct ecut_sectors {
    // model
    int32_t kind, cut_kind, n_sites;
    uint64_t left_mask;
    int32_t n_up, n_dn;
    std::vector<int> lsites, rsites;     // global site of each local bit
    // blocks
    std::vector<ecut::BlockDev> blocks;
    int64_t dim = 0;
    int32_t max_d_r = 0;
    // subsystem tables
    int32_t lcmin = 0, lcmax = -1, rcmin = 0, rcmax = -1;
    std::vector<int32_t> lcbase, rcbase;  // base of count c at [c - cmin]
    std::vector<uint32_t> lwords, rwords;
    std::vector<int32_t> hl_ptr, hl_col, hr_ptr, hr_col;
    std::vector<double> hl_val, hr_val, diag_l, diag_r;
    std::vector<ecut::XDiagDev> xdiag;
    std::vector<double> xdl;             // ProblemDev::xdl (empty: the terms one by one)
    std::vector<int32_t> xr_site;        // ProblemDev::xr_site
    std::vector<ecut::XBondDev> xbond;
    std::vector<int32_t> maps;
    int32_t n_cut_bonds = 0;
    bool hub_spatial = false;            // Hubbard model with a spatial cut (signed layout map)
    // Hubbard up/down kernel tables (host copies)
    bool hub_ok = false;
    bool hub2_ok = false;
    bool hub3_ok = false;                // fast class-tile kernel applies
    std::vector<int32_t> h3_seginfo, h3_loinfo, h3_looff, h3_hnb, h3_hcnt;
    int32_t h3_hs = 1, h3_max_tile = 0;
    ecut::Hub3Args h3{};                 // device pointers (launch fields filled per call)
    // segment-tile kernel
    bool hubseg_ok = false;
    std::vector<int32_t> hs_useg, hs_uhnb, hs_ulo, hs_ucross;
    std::vector<ecut::HubSegItem> hs_items;   // processing order, padded to 8 equal XCD chunks
    int32_t hs_uhs = 1, hs_n_slots = 0, hs_max_tile = 0;
    ecut::HubSegArgs hseg{};
    // two-pass flat kernels (variant 6): down-spin hops as slot-major ELL
    bool hub6_ok = false;
    std::vector<int32_t> level_rows;      // rows by inversion level (the left pass's row order)
    // the left operator's CSR with its rows in that order (row k = level_rows[k])
    std::vector<int32_t> h6_pptr, h6_pcol;
    std::vector<double> h6_pval;
    bool h6_uniform = false;              // every hop of either spin has the value h6_hop
    double h6_hop = 0.0;
    int32_t h6_maxq = 0;                  // bond slots of the down-spin table
    std::vector<int32_t> h6_col;
    std::vector<double> h6_val;
    ecut::HubUArgs h6u{};
    ecut::HubDArgs h6d{};
    ecut::HubDev hub{};
    std::vector<int32_t> hub_lo_cnt, hub_lo_ent, hub_lo_rank, hub_hi_cnt, hub_hi_ent, hub_seg_off, hub_xb;
    std::vector<double> hub_coef, hub_u;
    std::vector<uint16_t> hub_rw16;          // down word of each column (n <= 16)
    std::vector<uint32_t> hub_rw32;          // down word of each column
    std::vector<int32_t> hub_col_of_rank;    // column of the down word of canonical (colex) rank r
    std::vector<int32_t> hc_cls, hc_segcol, hc_hiw, hc_hicnt, hc_hient, hc_low, hc_locnt, hc_loent;
    std::vector<ecut::HubItem> hub_items;         // class-tile items, slot order
    std::vector<ecut::HubItem> hub_items_ord;     // class-tile items, processing order
    size_t hub_items_cap = 0;                     // device capacity for any processing order
    // Hubbard whole-row kernel (16-byte row access, hops ranked in LDS)
    bool hubrow_ok = false;
    std::vector<uint32_t> hrow_bmask, hrow_bbetw;
    std::vector<double> hrow_bcoef;
    // spin kernel with ranking tables
    bool spin_ok = false;
    std::vector<int32_t> spin_rank_lo, spin_rank_hi;
    std::vector<uint32_t> spin_fmask;
    std::vector<double> spin_fcoef;
    // work items of a single application (spin problems: may hold padding
    // items with row1 == row0 and slot -1)
    std::vector<ecut::ItemDev> items;
    size_t items_cap = 0;                 // device capacity for any spin tile size and order
    // two-pass spin kernels (variant 2): per-block level order of the left
    // words, the left pass's block table, one-row items at the head of `items`
    std::vector<int32_t> sp_level_rows;
    std::vector<int32_t> sp_pptr, sp_pcol;   // left operator's CSR in that order (per block, at lbase)
    std::vector<double> sp_pval;
    bool sp2_ok = false;                     // every left word has at most 64 neighbours
    // source columns of the right flip-flop terms and of the cross terms, per
    // block: right term f of column e at tbase[2b] + ((f / 4) * d_R + e) * 4 + f % 4,
    // cross term k at tbase[2b + 1] + k * d_R + e; 0xffff = no term
    std::vector<uint32_t> sp_rbetw;          // spatial Hubbard cut: bits between the two sites of each right hop
    std::vector<ecut::ItemDev> generic_items; // spatial Hubbard cut: the row kernel's items (variants 0, 1)
    std::vector<uint16_t> sp_tab;
    std::vector<int64_t> sp_tbase;
    const uint16_t *dev_sp_tab = nullptr;
    const int64_t *dev_sp_tbase = nullptr;
    std::vector<ecut::SpinLBlock> sp_lblocks;
    int32_t sp_n_one = 0;
    int32_t *dev_sp_rows = nullptr;
    const int32_t *dev_sp_pptr = nullptr, *dev_sp_pcol = nullptr;
    const double *dev_sp_pval = nullptr;
    ecut::SpinLBlock *dev_sp_lblocks = nullptr;
    int32_t item_slots = 0;               // partial-sum slots of `items` (its non-padding items)
    int32_t item_slots_cap = 0;           // most slots any spin tiling can use
    std::vector<int32_t> row_order;       // Hubbard kernel: row processing order
    int32_t kernel = 2;
    ecut::ApplyTuning tune{};
    // device side
    bool on_device = false;
    int device = -1;
    void *dev_mem = nullptr;
    size_t dev_bytes = 0;
    ecut::ProblemDev prob{};              // pointers into dev_mem
    ecut::ItemDev *dev_items = nullptr;
    int32_t *dev_row_order = nullptr;
    ecut::HubItem *dev_hub_items = nullptr;
    double n_eff = 0.0;
};

namespace ecut {
ecut_status build_host(const ecut_model_desc *m, const ecut_cut_desc *c, ecut_qnum q, ecut_sectors *s);
ecut_status upload(ecut_sectors *s);
void make_row_order(const ecut_sectors *s, int order, std::vector<int32_t> &out);
// row order used by work order `order` (0..10) of the Hubbard kernels
inline int row_order_kind(int order) { return order >= 9 ? 3 : order % 3; }
void make_hub_item_order(const ecut_sectors *s, int order, std::vector<HubItem> &out);
int32_t hub_column(const ecut_sectors *s, int64_t r);
// work items of the spin kernel for a short-row tile of `tile` amplitudes;
// order 0 largest first, 1 segments dealt to 8 XCD chunks (padded list);
// returns the number of partial-sum slots
int32_t make_spin_items(const ecut_sectors *s, int32_t tile, int32_t order, std::vector<ItemDev> &out);
// The left operator's CSR (hl_ptr / hl_col / hl_val) with its rows permuted:
// processing position p of a block takes the block's local row order[p]
// (positions and rows counted from the block's lbase); entries keep their
// order.  Returns the largest row length.
int32_t processing_csr(const ecut_sectors *s, const std::vector<int32_t> &order, std::vector<int32_t> &pptr,
                       std::vector<int32_t> &pcol, std::vector<double> &pval);
// left-pass block table of the two-pass spin kernels
void spin_left_blocks(const ecut_sectors *s, int32_t rows_per_item, std::vector<SpinLBlock> &out);
void release_device(ecut_sectors *s);
// item counts of the two-pass kernels (variant 6) for the handle's tuning
void hub6_shape(const ecut_sectors *s, HubUArgs &U, HubDArgs &D);
}  // namespace ecut
