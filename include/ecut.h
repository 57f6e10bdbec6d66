/*
 * ecut.h -- C ABI of libecut.so: the entanglement-cut bipartite Hamiltonian
 * application H*psi on MI355X (gfx950), the Lanczos ground-state solver built
 * on it, batched application over many sectors/Hamiltonians, and a
 * continuous-batching ground-state server.
 *
 * Problem statement (paper, Eq. 1-3):
 *   - H is K-local (K <= 2 here) on S sites with an Abelian symmetry Q
 *     (Eq. 1): U(1) Sz for spin-1/2 models, U(1)xU(1) (N_up, N_dn) for the
 *     Hubbard model;
 *   - an entanglement cut C splits the system into L and R with
 *     q_l (+) q_r = q, giving the blocks of Eq. (2);
 *   - the state is the set of block matrices Psi_q of Eq. (3), stored here
 *     row-major as Psi_q[l][r] (the paper's column-stacked Psi^q_{r l} is the
 *     same memory), blocks by ascending q_l, contiguous, no padding.
 *     Position of (q, l, r) = offset[q] + l * d_R[q] + r, where l and r are
 *     the colex ranks (= rank in increasing integer order) of the left and
 *     right subsystem words.  Exception: when the Hubbard up/down kernels
 *     apply (ecut_sectors_info.kernel == 1) the columns are in class-major
 *     order -- down words sorted by the popcount of their high half (sites
 *     n/2..n-1), then by the high half, then by the low half -- so that every
 *     class of down words closed under all hops but the one across n/2 is a
 *     contiguous run; ecut_sectors_words returns the down words in column
 *     order and ecut_canonical_positions gives the map.
 *
 * Conventions shared by every entry point:
 *   - Device pointers (suffix _d) are caller-owned device memory on the
 *     current HIP device; host pointers are caller-owned host memory.
 *     The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that take
 *     a stream are asynchronous on it unless stated otherwise.
 *   - Every call returns an ecut_status and never throws.  Argument errors
 *     are reported before any device work is queued.  A message for the last
 *     failure of the calling thread is available from ecut_last_error().
 *   - Apart from their launch tuning (ecut_set_tuning, ecut_autotune),
 *     handles are immutable after ecut_build_sectors and may be used from
 *     several streams and threads at once for ecut_apply_H.
 */
#ifndef ECUT_H
#define ECUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ECUT_OK = 0,
    ECUT_EINVAL = -1,        /* bad argument, null pointer, inconsistent model */
    ECUT_ENOMEM = -2,        /* host or device allocation failed / over budget */
    ECUT_EDEVICE = -3,       /* a HIP call failed (also asynchronous errors) */
    ECUT_ENOTCONV = -4,      /* Lanczos stopped at max_steps before tol */
    ECUT_EUNSUPPORTED = -5,  /* valid request outside what this build handles */
    ECUT_EAGAIN = -6         /* server: nothing finished yet */
} ecut_status;

enum { ECUT_SPIN_HALF = 1, ECUT_HUBBARD = 2 };
enum { ECUT_CUT_SPATIAL = 1, ECUT_CUT_UPDN = 2 };

/* Flags of ecut_build_sectors. */
enum {
    ECUT_BUILD_HOST_ONLY = 1   /* build host tables only; device calls then return ECUT_EINVAL */
};

/*
 * K-local Hamiltonian (Eq. 1) with K <= 2.
 *   ECUT_SPIN_HALF: H = sum_b jxy[b] (Sx_i Sx_j + Sy_i Sy_j) + jz[b] Sz_i Sz_j,
 *                   S = sigma/2, i = bond_i[b], j = bond_j[b]; site i = bit i
 *                   of the occupation word, spin up = bit set.  t, u unused.
 *   ECUT_HUBBARD:   H = -sum_b t[b] sum_s (c+_{i s} c_{j s} + h.c.)
 *                       + sum_i u[i] n_{i up} n_{i dn} + sum_b v[b] n_i n_j.
 *                   Fermion order: all up modes, then all down modes, each by
 *                   increasing site.  u may be NULL (all zero).  jxy, jz unused.
 * Arrays are read during ecut_build_sectors only.
 */
typedef struct ecut_model_desc {
    int32_t kind;             /* ECUT_SPIN_HALF | ECUT_HUBBARD */
    int32_t n_sites;          /* spin: 1..64; Hubbard: 1..32 */
    int32_t n_bonds;          /* >= 0 */
    int32_t reserved;         /* must be 0 */
    const int32_t *bond_i;    /* [n_bonds], 0 <= bond_i < n_sites */
    const int32_t *bond_j;    /* [n_bonds], bond_j != bond_i */
    const double *jxy;        /* [n_bonds] spin */
    const double *jz;         /* [n_bonds] spin */
    const double *t;          /* [n_bonds] Hubbard */
    const double *u;          /* [n_sites] Hubbard, nullable */
    const double *v;          /* [n_bonds] Hubbard: + v[b] n_i n_j with n = n_up + n_dn (the extended
                                 model); nullable; nonzero only with a spatial cut */
} ecut_model_desc;

/*
 * Entanglement cut C (paper, Fig. 1(a-c)).
 *   ECUT_CUT_SPATIAL (spin): L = sites whose bit is set in left_mask, R = the
 *       rest; subsystem word bit k = k-th site of that part in increasing
 *       site order.  Both parts need 1..32 sites.
 *   ECUT_CUT_SPATIAL (Hubbard, the real-space cut of Fig. 1(b)): L and R as
 *       above, at most 16 sites each; a subsystem word is (up << n) | dn
 *       over its n sites; blocks are (N_up_L, N_dn_L) in lexicographic order
 *       (ecut_sectors_labels), rows and columns the words of the block's
 *       numbers in increasing integer order.  The bipartite basis state
 *       |l, r> orders the creation operators of l's modes (up modes by site,
 *       then down modes) before r's, so the layout map carries a fermion
 *       sign (ecut_canonical_signs; ecut_import and ecut_export apply it).
 *       Hops across the cut are the sector-changing cross terms
 *       -t (c+_i (x) c_j + h.c.) with the left parity string, v[b] across
 *       the cut a diagonal cross term.  The generic row kernel applies it.
 *   ECUT_CUT_UPDN (Hubbard): the cut in the spin-group space of Fig. 1(c):
 *       L = up-spin occupation word, R = down-spin word; one block
 *       (N_up, N_dn); left_mask unused.  The Hubbard H then has the diagonal
 *       cross term U n_up n_dn only (the "particularly symmetric" case).
 */
typedef struct ecut_cut_desc {
    int32_t kind;
    int32_t reserved;         /* must be 0 */
    uint64_t left_mask;
} ecut_cut_desc;

/* Target sector q: spin: n_up = number of up spins (n_dn ignored);
 * Hubbard: particle numbers per spin species. */
typedef struct ecut_qnum {
    int32_t n_up;
    int32_t n_dn;
} ecut_qnum;

typedef struct ecut_sectors ecut_sectors;

typedef struct ecut_sectors_info {
    int64_t dim;              /* sum_q d_L[q] d_R[q] */
    int32_t n_blocks;         /* N_Q, blocks with d_L d_R > 0 */
    int32_t n_left_sites;
    int32_t n_right_sites;
    int32_t max_d_r;          /* longest block row */
    int32_t n_cut_bonds;      /* bonds with one end in L and one in R (spin) */
    int32_t n_cross_offdiag;  /* sector-changing L_m (x) R_m products (2 per cut bond with jxy != 0) */
    int32_t n_cross_diag;     /* diagonal cross-cut terms */
    int32_t kernel;           /* kernel family chosen for ecut_apply_H (1 = Hubbard up/down, 2 = generic rows) */
    int32_t kernel_flags;     /* Hubbard: bit 0 class tiles available, bit 1 uniform-chain fast path
                                 (and the split two-pass variant) available; spin: bit 2 the
                                 ranking-table kernel available (both parts <= 16 sites, row
                                 tiles <= 7168 amplitudes, <= 64 flip-flop terms in the right part);
                                 Hubbard: bit 3 the whole-row kernel available (<= 16 sites, even
                                 row length <= 14336, <= 64 bonds); bit 4 the segment-tile kernel
                                 available (as bit 1, and every tile fits 512 threads x 10
                                 slots and 48 KB of LDS); bit 5 the two-pass kernels available
                                 (at most 32 hopping bonds); spin and the spatial Hubbard cut:
                                 bit 6 the two-pass row kernels available (both parts <= 16
                                 sites, rows <= 6,656 amplitudes, <= 64 right terms and <= 64
                                 left-operator terms per row) */
    int32_t reserved;
    int64_t device_bytes;     /* device metadata held by the handle */
    double n_eff;             /* 1 / sum_q w_q^2 with w_q = d_L d_R / dim (block-size participation number) */
} ecut_sectors_info;

/*
 * Build the symmetry-resolved bipartite description of H for one sector:
 * subsystem bases with colex ranking, the block list (q_l + q_r = q, Eq. 2),
 * off-diagonal CSR of H_L and H_R per subsystem count, their diagonals, the
 * cross-cut diagonal terms and the sector-changing cross terms L_m (x) R_m
 * (partial permutations), then upload them to the current device.
 *   flags: ECUT_BUILD_HOST_ONLY to skip the device upload (host queries only).
 * Errors: ECUT_EINVAL (bad model/cut/qnum, e.g. a spin model with an
 * up/down cut or counts outside 0..sites, which would give an empty sector),
 * ECUT_EUNSUPPORTED (subsystem wider than 32 sites; Hubbard with a spatial
 * cut), ECUT_ENOMEM, ECUT_EDEVICE.  Synchronous.  *out owns its memory;
 * release it with ecut_sectors_free.
 */
ecut_status ecut_build_sectors(const ecut_model_desc *model, const ecut_cut_desc *cut,
                               ecut_qnum q, uint32_t flags, ecut_sectors **out);

void ecut_sectors_free(ecut_sectors *s);

ecut_status ecut_sectors_get_info(const ecut_sectors *s, ecut_sectors_info *info);

/* blocks: host int64 array of n_blocks x 5 entries (q_l, q_r, d_L, d_R, offset). */
ecut_status ecut_sectors_blocks(const ecut_sectors *s, int64_t *blocks);

/* Subsystem words of one block in row and column order: l_words[d_L],
 * r_words[d_R] (host arrays; either may be NULL).  Row and column order is
 * the colex rank, except for the class-major columns described above. */
ecut_status ecut_sectors_words(const ecut_sectors *s, int32_t block,
                               uint32_t *l_words, uint32_t *r_words);

/* pos[i] = bipartite position of the i-th sector state in canonical order
 * (full occupation words in increasing integer order; Hubbard word =
 * (up << n_sites) | dn).  Host array of dim entries.  Host only. */
ecut_status ecut_canonical_positions(const ecut_sectors *s, int64_t *pos);

/* sign[i] = +-1 with bip[pos[i]] = sign[i] * canon[i]: the parity of the
 * reordering of the i-th word's fermion modes from the canonical order to
 * the bipartite order (spatial Hubbard cut; +1 for every other problem).
 * Host array of dim entries.  Host only. */
ecut_status ecut_canonical_signs(const ecut_sectors *s, int8_t *sign);

/* labels: host int32 array of n_blocks x 4 entries (N_L, N_L2, N_R, N_R2):
 * the particle numbers of each block's two parts (spin models and the
 * up/down cut: N_L2 = N_R2 = 0 and N_L, N_R = q_l, q_r; spatial Hubbard cut:
 * up-spin and down-spin numbers). */
ecut_status ecut_sectors_labels(const ecut_sectors *s, int32_t *labels);

/* Permute a device vector between canonical order and the bipartite layout
 * (bip[pos[i]] = canon[i] and back).  In and out must not overlap. */
ecut_status ecut_import(const ecut_sectors *s, const double *canon_d, double *bip_d, void *stream);
ecut_status ecut_export(const ecut_sectors *s, const double *bip_d, double *canon_d, void *stream);

/*
 * y = H psi in the bipartite layout (Eq. 2 with the paper's local products,
 * its transposed left products and its cross terms evaluated in place):
 *   Y_q[l,:] = sum_l' H_L[l,l'] Psi_q[l',:]            (left operator, row combination)
 *            + Psi_q[l,:] H_R^T                        (right operator, in-row gather)
 *            + (d_L[l] + d_R[r] + diagonal cross terms) Psi_q[l,r]
 *            + sum_m A_m Psi_k B_m^T                    (sector-changing cross terms)
 * psi_d, y_d: dim doubles each, must not overlap; with the whole-row
 * Hubbard kernel (tuning variant 4) both must be 16-byte aligned (else
 * ECUT_EINVAL).  Asynchronous on stream.
 */
ecut_status ecut_apply_H(const ecut_sectors *s, const double *psi_d, double *y_d, void *stream);

/*
 * n independent applications y_k = H_k psi_k, the batched sector dispatch
 * over many Hamiltonians (the uneven symmetry sectors of the paper's
 * discussion of symmetry fragmentation, Eq. (3) blocks of every problem).
 * Spin and generic problems share one work queue over (problem, block, row
 * tile), largest tiles first (one launch of the spin kernel pair and/or one
 * of the generic row kernel); Hubbard up/down problems tuned to the two-pass
 * kernels (variant 6, at most 16 hopping bonds) share one launch per pass,
 * other Hubbard tunings run their own kernels.  Each output equals what
 * ecut_apply_H gives for that problem alone, bit for bit.
 * s, psi_d, y_d: host arrays of n entries.  The launch descriptors go
 * through device buffers the library allocates on first use and grows (a
 * ring of four per calling thread, with pinned staging): the call does not
 * wait for the device unless all four still hold descriptors of batches in
 * flight.  Asynchronous on stream otherwise.
 */
ecut_status ecut_apply_H_batch(int32_t n, const ecut_sectors *const *s, const double *const *psi_d,
                               double *const *y_d, void *stream);

/*
 * ecut_apply_H_batch for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * applications, launches and results (bit for bit) as ecut_apply_H_batch,
 * but the launch descriptors go into a fixed device array of the library
 * (ECUT_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends), written
 * by a small kernel on `stream` that carries them as kernel arguments: no
 * hipMalloc, hipFree or pinned host memory, and no wait on the host.  The
 * caller still owns psi_d and y_d.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * descriptors: calls on one GPU must be ordered (the same stream, or streams
 * the caller orders); calls that overlap on one GPU race.
 * Errors: as ecut_apply_H_batch; ECUT_EINVAL (before any device work) when
 * the batch's descriptors exceed ECUT_NOALLOC_SCRATCH_BYTES (problems with
 * many small work items, e.g. small spin tiles, take the most).
 */
#define ECUT_NOALLOC_SCRATCH_BYTES ((size_t)4 << 20)
ecut_status ecut_apply_H_batch_noalloc(int32_t n, const ecut_sectors *const *s, const double *const *psi_d,
                                       double *const *y_d, void *stream);

/*
 * Launch tuning of ecut_apply_H (used by the Hubbard up/down kernel, whose
 * work groups each own one row of Psi at a time):
 *   grid:      work groups (0 = one per compute unit);
 *   n_xcd:     rows are split into n_xcd contiguous chunks of the row order,
 *              chunk k served by the work groups with blockIdx % n_xcd == k
 *              (the accelerator complex that dispatches them), so rows that
 *              share neighbours share an L2 (0 = 8, 1 = plain grid stride);
 *   row_order: 0 increasing row index; 1 by inversion level of the left word
 *              (a nearest-neighbour hop changes it by exactly one, so all
 *              left-operator neighbours of a row sit in the adjacent levels);
 *              2 segment-major: rows grouped by the high half of the left
 *              word, groups ordered by the inversion level of that half;
 *              3..5: as 0..2 with the column classes of one row processed
 *              together instead of one class after the other;
 *              6..8: as 0..2, class major, with the row groups that share
 *              the high half of the up word dealt round-robin to the XCDs;
 *              9: rows sorted by the popcount of the high half of the left
 *              word, then by inversion level, class major (the source rows
 *              of one level then lie in a window of three levels that stays
 *              in the last-level cache); 10: as 9 with the classes of one
 *              row together;
 *   variant:   0 class tiles (rows cut into classes of down words, several
 *              work groups per CU; the uniform-chain fast kernel when it
 *              applies), 1 whole rows staged in LDS, 2 generic class tiles,
 *              3 two passes: the left operator over L2-resident column slabs,
 *              then the right operator and diagonal on class tiles,
 *              4 whole rows with 16-byte access: the row in LDS, down-spin
 *              hops found by ranking the hopped word (any hopping graph;
 *              needs kernel_flags bit 3 and 16-byte aligned vectors),
 *              5 segment tiles: (up segment) x (down segment) tiles, where a
 *              segment is the words sharing the high half, so hops inside
 *              either low half are read from LDS; the tiles of one panel
 *              (up segment x down class) run together on one XCD so the
 *              down high-half hops find their source in L2 (needs
 *              kernel_flags bit 4; row_order ignored; n_xcd 1 = plain grid
 *              stride, else 8 XCD chunks),
 *              6 two passes of one work group per item (kernel_flags bit 5):
 *              the left operator over column slabs in inversion-level row
 *              order (grid = rows per item, 0 = 4, at most 32), then the
 *              right operator, diagonal and epilogue with the source
 *              column of every hopping bond held in registers (tile = rows
 *              per item of that pass, 1, 2, 4, 8 or 16; 0 = 2); items dealt
 *              to the XCDs in contiguous ranges (n_xcd 1 = in launch order),
 *              7 the same left pass, then the right operator on class tiles
 *              (needs kernel_flags bit 1); tile = slabs side by side in one
 *              left-pass item (0 = 1, or 2 or 4; grid at most 32 / tile).
 *              Spin and generic problems (kernel 2) take variant 0 (the
 *              ranking-table spin kernel when kernel_flags bit 2 is set, else
 *              the generic row kernel) or 1 (the generic row kernel, which
 *              reads the right operator's CSR); n_xcd and row_order are
 *              ignored for them.  Spin problems also take variant 2: two
 *              passes, the left operator of every block over column slabs in
 *              inversion-level row order (grid = rows per item, 0 = 4, at
 *              most 32), then the spin kernel's right operator, cross terms,
 *              diagonal and epilogue starting from that sum, its one-row
 *              items grouped by the left sites no cross term touches (so a
 *              group's rows are each other's cross-term source rows);
 *              n_xcd 1 deals items in launch order, else in 8 contiguous
 *              XCD ranges; tile as for variant 0; the vector is variant
 *              0's bit for bit.  The spatial Hubbard cut (kernel 2,
 *              kernel_flags bit 6) takes variant 2 too: the same two passes
 *              with the fermion signs of hops inside the right part and
 *              across the cut, every row its own item (tile 0); its
 *              vector agrees with variant 0's to rounding;
 *   tile:      Hubbard variant 4: threads per work group, 256, 512 or 1024
 *              (0 = 1024); a row must fit 14 columns per thread (2 x 7
 *              column pairs), and smaller groups put more rows in flight on a
 *              CU.  For it, grid = work groups (0 = as many as fit on the
 *              device).  Every group size sums the terms of an amplitude in
 *              the same order, so the vector is the same bit for bit.
 *              Spin problems (kernel_flags bit 2): the work items of the
 *              sector queue are single rows for rows
 *              longer than tile/2 amplitudes, and runs of shorter rows of at
 *              most `tile` amplitudes otherwise (0 = 512, at most 512).
 *              Smaller tiles give more, smaller items; the Lanczos
 *              workspace (ecut_lanczos_workspace) holds the per-item partial
 *              sums of the smallest tile, so it does not change with tuning.
 *              Any other problem or variant takes tile 0.  For the spin kernel, grid is
 *              the number of work groups that stride through the item queue
 *              (0 = min(items, 2048)); the generic row kernel ignores it.
 * ecut_set_tuning re-uploads the row order or the work items (synchronous).
 * Not to be called while an ecut_apply_H on the same handle is in flight.
 * Results of different tunings agree to rounding (the terms of an amplitude
 * are summed in the same order by every spin tiling; the Lanczos partial sums
 * follow the item split).
 */
typedef struct ecut_tuning {
    int32_t grid;
    int32_t n_xcd;
    int32_t row_order;
    int32_t variant;
    int32_t tile;
} ecut_tuning;

ecut_status ecut_get_tuning(const ecut_sectors *s, ecut_tuning *t);
ecut_status ecut_set_tuning(ecut_sectors *s, const ecut_tuning *t);

/*
 * Autotuner: times ecut_apply_H(x_d -> y_d) for each candidate launch tuning
 * (Hubbard: kernel variant, row order, XCD chunking; spin: short-row tile and
 * grid, the generic row kernel, the two-pass kernels) with HIP events on `stream`, keeps the
 * fastest on the handle and returns it in *best (nullable).  x_d, y_d: dim
 * doubles each (contents of y_d are overwritten).  If the environment
 * variable ECUT_TUNE_CACHE names a JSON file, results are read from and
 * written to it, keyed by device architecture and problem shape.
 * Synchronous.
 */
ecut_status ecut_autotune(ecut_sectors *s, const double *x_d, double *y_d, void *stream, ecut_tuning *best);

/* Options of the Lanczos ground-state solver. */
typedef struct ecut_lanczos_opts {
    int32_t max_steps;        /* Krylov steps per restart cycle, >= 1 */
    int32_t max_restarts;     /* explicit restarts from the current Ritz vector (needs reorth) */
    int32_t reorth;           /* 0: three-term recurrence; 1: full reorthogonalisation (classical
                                 Gram-Schmidt, a second pass when the first removes over half the
                                 squared norm) */
    int32_t fixed_steps;      /* 1: run exactly max_steps (no convergence test) */
    double tol;               /* energy tolerance: stop when the lowest Ritz value moved by <= tol
                                 over the last step and its residual beta_j |s_j| <= 0.01 sqrt(tol)
                                 (the energy error of a Ritz value is of the order of the squared
                                 residual over the spectral gap) */
    int32_t use_graph;        /* 1: replay the steps of a three-term solve (after the first) from
                                 HIP graphs captured once per ring phase, so a step costs one graph
                                 launch on the host; 0: launch every kernel each step.  Same results
                                 bit for bit.  With the null stream the solve runs on a private
                                 stream ordered after the caller's work */
} ecut_lanczos_opts;

typedef struct ecut_lanczos_stats {
    int32_t steps;            /* steps in the tridiagonal matrix (one matvec each); with tol and
                                 no reorthogonalisation one more matvec runs after convergence
                                 and is not counted */
    int32_t restarts;
    int32_t converged;
    int32_t reserved;
    double residual;          /* last Ritz residual estimate */
    double seconds;           /* wall time of the solve */
} ecut_lanczos_stats;

/*
 * Lowest eigenvalue of H in this sector by Lanczos (the Krylov core the
 * paper's H*psi serves).  Per step: u = H v_j - beta_{j-1} v_{j-1} with
 * alpha_j = <v_j,u> fused into the H*psi kernel, w = u - alpha_j v_j,
 * optional reorthogonalisation against all stored vectors, beta_j = |w|; on
 * the host the lowest Ritz value is updated every step by Sturm bisection and
 * the returned energy is cross-checked by implicit QL on the final matrix.
 *   v0_d:    start vector (dim), not modified; must not be zero.
 *   basis_d: caller-owned device workspace of ecut_lanczos_workspace(s, opts)
 *            doubles.
 *   gs_d:    optional (nullable) output ground-state vector (dim); needs reorth=1.
 *   energy:  host output.  stats: nullable host output.
 * The factors of each step (1/beta_j for the next vector, beta_j s_j for the
 * previous one, with v_j = s_j w_j kept unnormalised) are computed on the
 * device.  Without reorthogonalisation two steps are in flight: the host
 * reads alpha_j, beta_j of step j (one small device-to-host copy per step)
 * while the device runs step j + 1, and drops that step if step j ends the
 * solve.  With reorthogonalisation one step is in flight (a restart may
 * follow).  Synchronises the stream before returning.
 * Returns ECUT_ENOTCONV (with energy set) if tol was not reached.
 */
size_t ecut_lanczos_workspace(const ecut_sectors *s, const ecut_lanczos_opts *opts);
ecut_status ecut_lanczos_ground_state(const ecut_sectors *s, const double *v0_d,
                                      const ecut_lanczos_opts *opts, double *energy,
                                      double *gs_d, ecut_lanczos_stats *stats,
                                      double *basis_d, void *stream);

/* ---------------------------------------------------------------------------
 * Krylov dynamical correlations: the one-particle Green's function from
 * Lanczos coefficients (the Krylov-based methods the paper names as the
 * users of H*Psi, in the discussion after Eq. (3)).
 *
 * ecut_apply_cdag: y = c+_{site,spin} x (dagger = 1) or c_{site,spin} x
 *   (dagger = 0) from sector src to sector dst of the same Hubbard lattice,
 *   both with the up/down cut; dst must hold src's particle numbers with one
 *   more (c+) or one fewer (c) of the given spin (0 = up, 1 = down).
 *   Fermion order as in ecut_model_desc (all up modes, then all down modes,
 *   each by site): the sign is (-1)^(occupied modes before the mode).  An up
 *   mode maps rows of src to rows of dst, a down mode columns to columns.
 *   x_d: src dim doubles; y_d: dst dim doubles (overwritten).  Asynchronous.
 *   Errors: ECUT_EINVAL (sectors that do not match), ECUT_EUNSUPPORTED
 *   (another model or cut).
 *
 * ecut_lanczos_tridiag: the Lanczos coefficients of H on the start vector
 *   v0_d / |v0_d|: n_steps three-term steps (fewer at an invariant subspace),
 *   alpha[j], beta[j] (beta[j] joins steps j and j + 1) into host arrays of
 *   n_steps entries, *n_out = steps taken, *v0_norm2 = |v0|^2 (nullable).
 *   basis_d: ecut_lanczos_workspace(s, {max_steps = n_steps, fixed_steps =
 *   1}) doubles.  Synchronous.  Errors: ECUT_EINVAL (v0 zero: *v0_norm2 is
 *   then 0), as ecut_lanczos_ground_state.
 *
 * ecut_continued_fraction: G(w) at n_omega frequencies (host arrays):
 *   dagger = 1: G+(w) = weight / (z - a0 - b0^2 / (z - a1 - b1^2 / ...)),
 *               z = w + i eta + e0;
 *   dagger = 0: G-(w) = weight / (z + a0 - b0^2 / (z + a1 - ...)),
 *               z = w + i eta - e0;
 *   with the coefficients of H on c+ psi0 (resp. c psi0), weight = the
 *   squared norm of that vector and e0 the ground energy of psi0, so that
 *   G+(w) = <psi0| c (w + i eta + e0 - H)^-1 c+ |psi0> and
 *   G-(w) = <psi0| c+ (w + i eta - e0 + H)^-1 c |psi0>.  Host only.
 * ------------------------------------------------------------------------- */
ecut_status ecut_apply_cdag(const ecut_sectors *src, const ecut_sectors *dst, int32_t site, int32_t spin,
                            int32_t dagger, const double *x_d, double *y_d, void *stream);
ecut_status ecut_lanczos_tridiag(const ecut_sectors *s, const double *v0_d, int32_t n_steps, double *alpha,
                                 double *beta, int32_t *n_out, double *v0_norm2, double *basis_d, void *stream);
ecut_status ecut_continued_fraction(const double *alpha, const double *beta, int32_t n, double weight, double e0,
                                    int32_t dagger, const double *omega, int32_t n_omega, double eta, double *g_re,
                                    double *g_im);

/* ---------------------------------------------------------------------------
 * Entanglement spectrum of a state (the paper's discussion of the
 * distributed entanglement spectrum, with its figure of xi_{q,i} over the
 * sectors and the process-resolved W_P, and the End Matter's N_eff).
 *   rho_L = Tr_R |psi><psi| / <psi|psi> is block diagonal over the blocks of
 *   the cut; lambda_{q,i} are the eigenvalues of block q (the squared
 *   Schmidt values, min(d_L, d_R) of them per block, descending), and
 *   xi_{q,i} = -log lambda_{q,i} the spectrum of H_E = -log rho_L.
 *   W_q = sum_i lambda_{q,i} (the entanglement weight of sector q);
 *   W_P[p] = sum_{q in Q_p} W_q^2 over the sectors assigned to part p
 *   (part_of_block, or when NULL a largest-first packing of the blocks by
 *   dimension into n_parts parts, the sector sharding of this build);
 *   chi_q = number of lambda_{q,i} above `cutoff` (the sector's Schmidt
 *   rank), n_eff = 1 / sum_q (chi_q / sum chi)^2 (the End Matter's
 *   participation number of the sector dimensions), weight_ipr =
 *   1 / sum_q W_q^2, entropy = -sum lambda log lambda.
 * Per block the Gram matrix of the smaller side (Psi_q Psi_q^T or
 * Psi_q^T Psi_q) is formed with rocBLAS syrk, and the blocks whose Gram
 * matrices have one size are diagonalised together with rocSOLVER's batched
 * syevd, on the device; the rest on the host.
 *   psi_d:       state in the bipartite layout (dim doubles, any norm, not 0).
 *   workspace_d: ecut_entanglement_sizes(s, &n_lambda) doubles (device).
 *   lambda, xi:  host, n_lambda doubles each, blocks in order (xi nullable;
 *                +inf where lambda <= 0).
 *   w_q, chi_q:  host, n_blocks entries; w_p: host, n_parts (nullable if
 *                n_parts == 1).
 * Synchronises the stream.  Errors: ECUT_EINVAL (null or bad arguments, zero
 * state), ECUT_ENOTCONV (the eigensolver did not converge), ECUT_EDEVICE.
 * ------------------------------------------------------------------------- */
typedef struct ecut_entanglement {
    int32_t n_blocks;
    int32_t n_parts;
    int64_t n_lambda;
    double norm2;             /* <psi|psi> */
    double weight_ipr;        /* 1 / sum_q W_q^2 */
    double n_eff;             /* 1 / sum_q (chi_q / sum chi)^2 */
    double entropy;           /* -sum lambda log lambda */
} ecut_entanglement;

size_t ecut_entanglement_sizes(const ecut_sectors *s, size_t *n_lambda);
ecut_status ecut_entanglement_spectrum(const ecut_sectors *s, const double *psi_d, double cutoff, int32_t n_parts,
                                       const int32_t *part_of_block, double *lambda, double *xi, double *w_q,
                                       int32_t *chi_q, double *w_p, ecut_entanglement *summary,
                                       double *workspace_d, void *stream);

/* ---------------------------------------------------------------------------
 * Continuous-batching ground-state server.
 * A worker thread owns one stream and a device arena of hbm_budget bytes;
 * a helper thread builds the sector tables of arrived requests (up to 16
 * ahead of the queue head, in arrival order) and frees those of retired
 * solves.  Requests are admitted when their footprint (sector metadata + Lanczos
 * vectors) fits the free arena and a slot is free; all admitted solves
 * advance together, one batched H*psi launch and one batched vector-update
 * launch per step, with two steps in flight (the host checks the solves of
 * step j while the device runs step j + 1); a solve leaves the batch when
 * converged (tol) or at max_steps, freeing its memory for the next admission
 * once no step of it is in flight.
 * ------------------------------------------------------------------------- */
typedef struct ecut_server ecut_server;

typedef struct ecut_server_opts {
    int32_t max_active;       /* slots; 0 = unlimited */
    int32_t max_steps;        /* per request */
    double tol;               /* energy tolerance per request (as ecut_lanczos_opts.tol) */
    int32_t sequential;       /* 1: one request at a time (max_active forced to 1), the
                                 one-at-a-time baseline on the same engine */
    int32_t use_graph;        /* 1: while the set of active solves stays the same, replay each
                                 batched step from a HIP graph captured once per ring phase (a new
                                 set drops the graphs); 0: launch every kernel each step.  Same
                                 results bit for bit */
    int32_t autotune;         /* 1: the first request of each problem shape (device architecture,
                                 sites, particle numbers, blocks, dimension) is autotuned on its own
                                 workspace (ecut_autotune); the tuning is kept for the life of the
                                 process and applied to every later request of that shape, in any
                                 server.  0: default launch tuning */
    int64_t large_dim;        /* > 0 (and not sequential): requests of at least this many amplitudes
                                 run on a second worker with its own stream, one at a time with
                                 the tuning for a problem alone, while the others batch on the
                                 first worker (max_active applies there); the two streams'
                                 kernels overlap on the device and share the arena.  Admission
                                 is FIFO within each lane, and no request takes arena space
                                 ahead of an earlier one of the other lane that waits for it.
                                 A large request then never shares its steps with the small
                                 ones that arrive meanwhile.  Not with use_graph (ECUT_EINVAL).
                                 0: one worker */
} ecut_server_opts;

typedef struct ecut_result {
    uint64_t req_id;
    int32_t status;           /* ecut_status of the solve */
    int32_t steps;
    double energy;
    double residual;
    double t_submit;          /* seconds on the server clock */
    double t_admit;
    double t_done;
} ecut_result;

ecut_status ecut_server_create(size_t hbm_budget, const ecut_server_opts *opts, ecut_server **out);

/* Queue one request.  not_before: earliest admission time on the server
 * clock (seconds since create; <= 0 = now).  The start vector is drawn on the
 * device directly in the bipartite layout: entry i is a Box-Muller normal from
 * two splitmix64 values of (seed, 2i) and (seed, 2i+1), so a request gets the
 * same vector alone or in a mix.  The model arrays are copied.  Thread-safe. */
ecut_status ecut_server_submit(ecut_server *srv, const ecut_model_desc *model, const ecut_cut_desc *cut,
                               ecut_qnum q, uint64_t seed, double not_before, uint64_t *req_id);

/* Copy up to max finished results; *n_done = number copied (0 -> ECUT_EAGAIN). */
ecut_status ecut_server_poll(ecut_server *srv, ecut_result *out, int32_t max, int32_t *n_done);

/* Block until every submitted request has finished.  A failure of the
 * server's own threads (not of a single request) is returned here and by
 * ecut_server_poll, with the worker's message in ecut_last_error(). */
ecut_status ecut_server_drain(ecut_server *srv);

/* Server clock (seconds since create). */
double ecut_server_now(const ecut_server *srv);

void ecut_server_destroy(ecut_server *srv);

/* Message of the last failed call on this thread ("" if none). */
const char *ecut_last_error(void);

/* Library version string. */
const char *ecut_version(void);

/* ---------------------------------------------------------------------------
 * Device memory for the sector tables.
 * Each handle keeps its tables (basis words, operator CSR, work lists, rank
 * tables) in one block of device memory the library allocates, with
 * hipMalloc unless the caller installs an allocator here: for instance one
 * backed by torch's caching allocator, so that the tables share its pool.
 *   alloc(bytes, device, user): at least `bytes` of device memory on HIP
 *     device `device` (the current device at the call), 256-byte aligned, or
 *     NULL.  NULL fails the building call with ECUT_ENOMEM; a misaligned
 *     block is handed back to free and the call fails with ECUT_EINVAL.
 *   free(ptr, bytes, device, user): releases a block alloc returned.  The
 *     library synchronises the device first, so no kernel still reads it.
 * Each block is released through the pair that made it: the pair may be
 * replaced at any time, but must stay callable while any block it made is
 * alive.  Both may be called from any thread, including the server's own.
 * Passing NULL, NULL restores hipMalloc / hipFree.  Not covered: the
 * server's arena (one hipMalloc of hbm_budget at create), the library's
 * per-device constant tables (kept until the process ends), its
 * launch-descriptor buffers (kept per thread and per server), and the
 * caller's own vectors and workspaces.
 * Errors: ECUT_EINVAL if exactly one of alloc and free is NULL.
 * ------------------------------------------------------------------------- */
typedef void *(*ecut_alloc_fn)(size_t bytes, int32_t device, void *user);
typedef void (*ecut_free_fn)(void *ptr, size_t bytes, int32_t device, void *user);
ecut_status ecut_set_allocator(ecut_alloc_fn alloc, ecut_free_fn free_fn, void *user);

#ifdef __cplusplus
}
#endif
#endif /* ECUT_H */
