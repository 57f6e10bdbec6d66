// Entanglement spectrum of a state in the bipartite layout: the spectrum
// xi_{q,i} = -log lambda_{q,i} of the entanglement Hamiltonian
// H_E = -log rho_L, rho_L = Tr_R |psi><psi| (the paper's figure on the
// distributed entanglement spectrum).  rho_L is block diagonal over the
// sectors of the cut, rho_L^q = Psi_q Psi_q^T, and its nonzero eigenvalues
// are those of the smaller Gram matrix of the block, Psi_q Psi_q^T or
// Psi_q^T Psi_q.  Per block: the Gram matrix with rocBLAS syrk (a plain
// dense contraction), its eigenvalues with rocSOLVER syevd, both on the
// device; the sector weights W_q, their participation numbers and the
// process-resolved sums W_P on the host.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "ecut_internal.h"
#include "runtime.h"

using namespace ecut;

namespace {

// one rocBLAS handle per thread and device
ecut_status blas_handle(rocblas_handle *h) {
    static thread_local std::map<int, rocblas_handle> handles;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(ECUT_EDEVICE, "hipGetDevice");
    auto it = handles.find(dev);
    if (it == handles.end()) {
        rocblas_handle nh = nullptr;
        if (rocblas_create_handle(&nh) != rocblas_status_success) return fail(ECUT_EDEVICE, "rocblas_create_handle");
        it = handles.emplace(dev, nh).first;
    }
    *h = it->second;
    return ECUT_OK;
}

int64_t schmidt_count(const ecut_sectors *s) {
    int64_t n = 0;
    for (const BlockDev &B : s->blocks) n += std::min(B.d_l, B.d_r);
    return n;
}

// parts of a largest-first bin packing of the blocks by dimension
std::vector<int32_t> pack_blocks(const ecut_sectors *s, int32_t n_parts) {
    std::vector<int32_t> order(s->blocks.size()), part(s->blocks.size(), 0);
    std::iota(order.begin(), order.end(), 0);
    auto dimq = [&](int32_t q) { return (int64_t)s->blocks[q].d_l * s->blocks[q].d_r; };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return dimq(a) > dimq(b); });
    std::vector<int64_t> load(n_parts, 0);
    for (int32_t q : order) {
        const int32_t p = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        part[q] = p;
        load[p] += dimq(q);
    }
    return part;
}

// the blocks by the size of their Gram matrix (m = min(d_L, d_R) > 0), in
// block order inside each size
std::map<int, std::vector<int32_t>> gram_groups(const ecut_sectors *s) {
    std::map<int, std::vector<int32_t>> g;
    for (int32_t q = 0; q < (int32_t)s->blocks.size(); ++q) {
        const int m = std::min(s->blocks[q].d_l, s->blocks[q].d_r);
        if (m > 0) g[m].push_back(q);
    }
    return g;
}

}  // namespace

extern "C" {

// Workspace: the Gram matrices of the largest group of equal-size blocks,
// the eigenvalues of every block, the eigensolver's off-diagonals for that
// group, one status word per block.
size_t ecut_entanglement_sizes(const ecut_sectors *s, size_t *n_lambda) {
    if (!s) return 0;
    size_t g_max = 0, e_max = 0;
    for (const auto &kv : gram_groups(s)) {
        const size_t m = (size_t)kv.first, c = kv.second.size();
        g_max = std::max(g_max, c * m * m);
        e_max = std::max(e_max, c * m);
    }
    const size_t nl = (size_t)schmidt_count(s);
    if (n_lambda) *n_lambda = nl;
    return g_max + nl + e_max + (s->blocks.size() + 1) / 2 + 1;
}

ecut_status ecut_entanglement_spectrum(const ecut_sectors *s, const double *psi_d, double cutoff, int32_t n_parts,
                                       const int32_t *part_of_block, double *lambda, double *xi, double *w_q,
                                       int32_t *chi_q, double *w_p, ecut_entanglement *summary, double *workspace_d,
                                       void *stream) {
    if (!s || !psi_d || !workspace_d || !lambda || !w_q || !chi_q || !summary)
        return fail(ECUT_EINVAL, "null argument");
    if (!s->on_device) return fail(ECUT_EINVAL, "handle was built with ECUT_BUILD_HOST_ONLY");
    if (n_parts < 1 || (n_parts > 1 && !w_p)) return fail(ECUT_EINVAL, "n_parts must be >= 1 (and w_p set)");
    if (!(cutoff >= 0.0)) return fail(ECUT_EINVAL, "cutoff must be >= 0");
    const int32_t nb = (int32_t)s->blocks.size();
    if (part_of_block)
        for (int32_t q = 0; q < nb; ++q)
            if (part_of_block[q] < 0 || part_of_block[q] >= n_parts) return fail(ECUT_EINVAL, "part_of_block out of range");
    for (const BlockDev &B : s->blocks)
        if (std::min(B.d_l, B.d_r) > (1 << 24)) return fail(ECUT_EUNSUPPORTED, "block too large for the Gram matrix");
    rocblas_handle h = nullptr;
    ecut_status st = blas_handle(&h);
    if (st != ECUT_OK) return st;
    const hipStream_t hs = (hipStream_t)stream;
    if (rocblas_set_stream(h, hs) != rocblas_status_success) return fail(ECUT_EDEVICE, "rocblas_set_stream");
    const auto groups = gram_groups(s);
    size_t g_max = 0;
    for (const auto &kv : groups) g_max = std::max(g_max, kv.second.size() * (size_t)kv.first * (size_t)kv.first);
    const int64_t n_lam = schmidt_count(s);
    // per group of equal-size blocks: their Gram matrices side by side
    // (rocBLAS syrk each), one batched eigensolve; the eigenvalues of every
    // group side by side, one copy to the host at the end
    double *G = workspace_d, *Dg = workspace_d + g_max, *E = Dg + n_lam;
    size_t e_max = 0;
    for (const auto &kv : groups) e_max = std::max(e_max, kv.second.size() * (size_t)kv.first);
    rocblas_int *info = (rocblas_int *)(E + e_max);
    const double one = 1.0, zero = 0.0;
    int64_t goff = 0;
    int32_t ioff = 0;
    for (const auto &kv : groups) {
        const int m = kv.first;
        const int c = (int)kv.second.size();
        for (int i = 0; i < c; ++i) {
            const BlockDev &B = s->blocks[kv.second[i]];
            // Psi_q is row-major d_L x d_R: column-major it is A (d_R x d_L, lda = d_R)
            const double *A = psi_d + B.offset;
            const bool left = B.d_l <= B.d_r;   // Psi Psi^T = A^T A (d_L x d_L), else Psi^T Psi = A A^T
            rocblas_status rs =
                rocblas_dsyrk(h, rocblas_fill_upper, left ? rocblas_operation_transpose : rocblas_operation_none, m,
                              left ? B.d_r : B.d_l, &one, A, B.d_r, &zero, G + (size_t)i * m * m, m);
            if (rs != rocblas_status_success) return fail(ECUT_EDEVICE, "rocblas_dsyrk: status " + std::to_string((int)rs));
        }
        const rocblas_status rs = rocsolver_dsyevd_strided_batched(h, rocblas_evect_none, rocblas_fill_upper, m, G, m,
                                                                   (rocblas_stride)m * m, Dg + goff, m, E, m,
                                                                   info + ioff, c);
        if (rs != rocblas_status_success)
            return fail(ECUT_EDEVICE, "rocsolver_dsyevd_strided_batched: status " + std::to_string((int)rs));
        goff += (int64_t)c * m;
        ioff += c;
    }
    std::vector<double> ev((size_t)n_lam);
    std::vector<rocblas_int> inf((size_t)std::max(ioff, 1), 0);
    hipError_t e = n_lam ? hipMemcpyAsync(ev.data(), Dg, sizeof(double) * n_lam, hipMemcpyDeviceToHost, hs) : hipSuccess;
    if (e == hipSuccess && ioff)
        e = hipMemcpyAsync(inf.data(), info, sizeof(rocblas_int) * ioff, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail(ECUT_EDEVICE, std::string("entanglement spectrum: ") + hipGetErrorString(e));
    // each block's eigenvalues, descending, at its place in block order
    std::vector<int64_t> lam_off((size_t)nb + 1, 0);
    for (int32_t q = 0; q < nb; ++q)
        lam_off[q + 1] = lam_off[q] + std::min(s->blocks[q].d_l, s->blocks[q].d_r);
    goff = 0;
    ioff = 0;
    for (const auto &kv : groups) {
        const int m = kv.first;
        for (size_t i = 0; i < kv.second.size(); ++i, ++ioff) {
            const int32_t q = kv.second[i];
            if (inf[ioff] != 0) return fail(ECUT_ENOTCONV, "rocsolver_dsyevd did not converge on block " + std::to_string(q));
            for (int k = 0; k < m; ++k) lambda[lam_off[q] + k] = ev[(size_t)(goff + (int64_t)i * m + m - 1 - k)];
        }
        goff += (int64_t)kv.second.size() * m;
    }
    int64_t off_l = n_lam;
    // normalise to the state's norm: the eigenvalues of rho_L of psi / |psi|
    const double norm2 = std::accumulate(lambda, lambda + off_l, 0.0);
    if (!(norm2 > 0.0)) return fail(ECUT_EINVAL, "the state is zero");
    off_l = 0;
    int64_t chi_sum = 0;
    double w2 = 0.0;
    for (int32_t q = 0; q < nb; ++q) {
        const BlockDev &B = s->blocks[q];
        const int m = std::min(B.d_l, B.d_r);
        double wq = 0.0;
        int32_t chi = 0;
        for (int i = 0; i < m; ++i) {
            double &l = lambda[off_l + i];
            l /= norm2;
            wq += l;
            if (l > cutoff) ++chi;
            if (xi) xi[off_l + i] = l > 0.0 ? -std::log(l) : INFINITY;
        }
        w_q[q] = wq;
        chi_q[q] = chi;
        chi_sum += chi;
        w2 += wq * wq;
        off_l += m;
    }
    double c2 = 0.0;
    for (int32_t q = 0; q < nb; ++q) {
        const double c = chi_sum > 0 ? (double)chi_q[q] / (double)chi_sum : 0.0;
        c2 += c * c;
    }
    std::vector<int32_t> part = part_of_block ? std::vector<int32_t>(part_of_block, part_of_block + nb)
                                              : pack_blocks(s, n_parts);
    if (w_p) {
        std::fill(w_p, w_p + n_parts, 0.0);
        for (int32_t q = 0; q < nb; ++q) w_p[part[q]] += w_q[q] * w_q[q];
    }
    ecut_entanglement S{};
    S.n_blocks = nb;
    S.n_parts = n_parts;
    S.n_lambda = off_l;
    S.norm2 = norm2;
    S.weight_ipr = w2 > 0.0 ? 1.0 / w2 : 0.0;
    S.n_eff = c2 > 0.0 ? 1.0 / c2 : 0.0;
    S.entropy = 0.0;
    for (int64_t i = 0; i < off_l; ++i)
        if (lambda[i] > 0.0) S.entropy -= lambda[i] * std::log(lambda[i]);
    *summary = S;
    return ECUT_OK;
}

}  // extern "C"
