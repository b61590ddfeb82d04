// Reduction kernels for gfx950: measurement probabilities (QCLAB section
// 3.3), Pauli-string expectation values and the state-difference report.
//
// All sums accumulate in FP64 whatever the state precision.  Every
// reduction is deterministic: a fixed grid, a fixed per-thread order, a
// wavefront butterfly (64 lanes) and a fixed cross-wave order inside each
// block, then a second pass that adds the per-block partials in block
// order.  No floating-point atomics are used anywhere.
#include "qc_internal.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum in a fixed order; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kWaves; ++w) r += lds[w];
    return r;
}
__device__ inline double block_max(double v, double *lds) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kWaves; ++w) r = fmax(r, lds[w]);
    return r;
}

template <typename R>
__device__ inline double norm2(cx<R> a) {
    const double re = double(a.re), im = double(a.im);
    return re * re + im * im;
}

// ---- probabilities -------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs_full(const cx<R> *amp, uint64_t count,
                                                       double *out) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride)
        out[i] = norm2(amp[i]);
}

struct PermArgs {
    uint32_t src_pos[QC_MAX_QUBITS];  // bit position of the qubit that becomes
                                      // outcome bit (m-1-j), j = list index
    int m;
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_probs_perm(const cx<R> *amp, uint64_t count,
                                                       const PermArgs p, double *out) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        uint64_t s = 0;
        for (int j = 0; j < p.m; ++j) s = (s << 1) | ((i >> p.src_pos[j]) & 1);
        out[s] = norm2(amp[i]);
    }
}

struct MarginalArgs {
    uint64_t bin_off[24];      // offset of outcome bit (m-1-j) = listed qubit j
    uint32_t pos[QC_MAX_QUBITS];  // ascending positions of the listed qubits
    int m;
    uint64_t rest;             // 2^(n-m) indices per bin
    uint64_t chunk;            // indices of one bin summed by one block
    int chunks;                // blocks per bin
    uint64_t items;            // bins * chunks
};

// Block (bin s, chunk c) sums |psi|^2 over its share of the bin's indices.
// Each thread keeps kMargLoads independent loads in flight.  With PAIR
// (complex64, bit 0 not a listed qubit) a load moves the two neighbouring
// amplitudes of indices r and r + 1 (16 bytes); complex128 amplitudes are
// 16 bytes each already.
constexpr int kMargLoads = 4;
typedef float floatx4_r __attribute__((ext_vector_type(4)));

template <typename R, bool PAIR>
__device__ inline void marginal_item(const cx<R> *amp, const MarginalArgs &a, uint64_t b,
                                     double *work, double *lds) {
    const uint64_t s = b / unsigned(a.chunks);
    const uint64_t c = b % unsigned(a.chunks);
    uint64_t binbase = 0;
    for (int j = 0; j < a.m; ++j)
        if ((s >> (a.m - 1 - j)) & 1) binbase |= a.bin_off[j];
    const uint64_t r0 = c * a.chunk;
    uint64_t r1 = r0 + a.chunk;
    if (r1 > a.rest) r1 = a.rest;
    constexpr uint64_t step = PAIR ? 2 : 1;
    double acc = 0.0;
    for (uint64_t r = r0 + step * threadIdx.x; r < r1; r += step * kBlock * kMargLoads) {
        if constexpr (PAIR) {
            floatx4_r v[kMargLoads];
#pragma unroll
            for (int u = 0; u < kMargLoads; ++u) {
                const uint64_t rr = r + u * step * kBlock;
                v[u] = floatx4_r{0.f, 0.f, 0.f, 0.f};
                if (rr < r1)
                    v[u] = *reinterpret_cast<const floatx4_r *>(amp + (insert_zeros(rr, a.pos, a.m) | binbase));
            }
#pragma unroll
            for (int u = 0; u < kMargLoads; ++u)
                acc += (double(v[u][0]) * double(v[u][0]) + double(v[u][1]) * double(v[u][1])) +
                       (double(v[u][2]) * double(v[u][2]) + double(v[u][3]) * double(v[u][3]));
        } else {
            cx<R> v[kMargLoads];
#pragma unroll
            for (int u = 0; u < kMargLoads; ++u) {
                const uint64_t rr = r + u * kBlock;
                v[u] = cx<R>{R(0), R(0)};
                if (rr < r1) v[u] = amp[insert_zeros(rr, a.pos, a.m) | binbase];
            }
#pragma unroll
            for (int u = 0; u < kMargLoads; ++u) acc += norm2(v[u]);
        }
    }
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) work[b] = tot;
}

// Work item b = (bin s, chunk c) = (b / chunks, b % chunks), b < items;
// blocks step through the items with a stride of the grid size (a launch
// may not hold more than 2^32 threads: 2^24 one-block bins exceed it).
template <typename R, bool PAIR>
__global__ __launch_bounds__(kBlock) void k_probs_marginal(const cx<R> *amp,
                                                           const MarginalArgs a, double *work) {
    __shared__ double lds[kWaves];
    for (uint64_t b = blockIdx.x; b < a.items; b += gridDim.x)
        marginal_item<R, PAIR>(amp, a, b, work, lds);
}

// out[s] = sum over the chunks of bin s, in chunk order.
__global__ __launch_bounds__(kBlock) void k_sum_rows(const double *work, int rows, int cols,
                                                     double *out) {
    __shared__ double lds[kWaves];
    const int row = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < cols; c += kBlock) acc += work[size_t(row) * cols + c];
    const double tot = block_sum(acc, lds);
    if (threadIdx.x == 0) out[row] = tot;
}

// ---- Pauli expectation -----------------------------------------------------
//
// For P = i^ny X^x Z^z (x, z bit masks, ny = number of Y factors):
//   P|j> = i^ny (-1)^popc(j & z) |j ^ x>,
//   <psi|P|psi> = sum_j i^ny (-1)^popc(j & z) conj(psi_{j^x}) psi_j.
// One launch serves all terms that share the same x mask.  With x != 0 a
// work item owns the pair (j, j ^ x), j having a zero at the top bit of x,
// and adds both contributions, so every amplitude is read exactly once.

struct ExpectArgs {
    uint64_t xmask;
    uint64_t n_items;
    uint64_t zmask[kExpectMaxTerms];
    int phase[kExpectMaxTerms];  // ny mod 4
    int hpos;                    // top bit of xmask, -1 if xmask == 0
    int n_terms;
};

// NT = the group's term count rounded up to 1, 4, 8, 16 or 32: the
// accumulators and the term tables are indexed with constants only, so they
// stay in registers.
template <typename R, int NT>
__global__ __launch_bounds__(kBlock) void k_expect_group(const cx<R> *amp, const ExpectArgs a,
                                                         double *work) {
    __shared__ double lds[kWaves];
    double acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < a.n_items; g += stride) {
        if (a.hpos < 0) {
            const double w = norm2(amp[g]);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (t < a.n_terms) acc[t] += (__popcll(g & a.zmask[t]) & 1) ? -w : w;
        } else {
            const uint64_t j = insert_zero(g, a.hpos);
            const uint64_t jx = j ^ a.xmask;
            const cx<R> pa = amp[j], pb = amp[jx];
            // conj(b) * a = c1 + i c2
            const double ar = pa.re, ai = pa.im, br = pb.re, bi = pb.im;
            const double c1 = br * ar + bi * ai;
            const double c2 = br * ai - bi * ar;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t < a.n_terms) {
                    const double sj = (__popcll(j & a.zmask[t]) & 1) ? -1.0 : 1.0;
                    const double sx = (__popcll(jx & a.zmask[t]) & 1) ? -1.0 : 1.0;
                    // i^ny * (sj conj(b) a + sx conj(a) b), real part
                    double v;
                    switch (a.phase[t]) {
                    case 0: v = (sj + sx) * c1; break;
                    case 1: v = -(sj - sx) * c2; break;
                    case 2: v = -(sj + sx) * c1; break;
                    default: v = (sj - sx) * c2; break;
                    }
                    acc[t] += v;
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
        if (t < a.n_terms) {   // uniform
            const double tot = block_sum(acc[t], lds);
            if (threadIdx.x == 0) work[size_t(t) * gridDim.x + blockIdx.x] = tot;
        }
}

// tab[t] = coefficient of term t, tab[n_terms + t] = slot of term t in vals
__global__ void k_expect_combine(const double *vals, const double *tab, int n_terms,
                                 int per_term, double *out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double e = 0.0;
    for (int t = 0; t < n_terms; ++t) {
        const double v = vals[int(tab[n_terms + t])];
        e += tab[t] * v;
        if (per_term) out[1 + t] = v;
    }
    out[0] = e;
}

// ---- state difference ------------------------------------------------------

template <typename RA, typename RB>
__global__ __launch_bounds__(kBlock) void k_diff(const cx<RA> *a, const cx<RB> *b,
                                                 uint64_t count, double *work) {
    __shared__ double lds[kWaves];
    double d2 = 0.0, b2 = 0.0, dm = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        const cx<RA> x = a[i];
        const cx<RB> y = b[i];
        const double dr = double(x.re) - double(y.re), di = double(x.im) - double(y.im);
        const double dd = dr * dr + di * di;
        d2 += dd;
        b2 += double(y.re) * double(y.re) + double(y.im) * double(y.im);
        dm = fmax(dm, dd);
    }
    const double t0 = block_sum(d2, lds);
    if (threadIdx.x == 0) work[blockIdx.x] = t0;
    const double t1 = block_sum(b2, lds);
    if (threadIdx.x == 0) work[gridDim.x + blockIdx.x] = t1;
    const double t2 = block_max(dm, lds);
    if (threadIdx.x == 0) work[2 * gridDim.x + blockIdx.x] = t2;
}

__global__ __launch_bounds__(kBlock) void k_diff_final(const double *work, int blocks,
                                                       double *out) {
    __shared__ double lds[kWaves];
    double s0 = 0.0, s1 = 0.0, mx = 0.0;
    for (int c = threadIdx.x; c < blocks; c += kBlock) {
        s0 += work[c];
        s1 += work[blocks + c];
        mx = fmax(mx, work[2 * blocks + c]);
    }
    const double t0 = block_sum(s0, lds);
    const double t1 = block_sum(s1, lds);
    const double t2 = block_max(mx, lds);
    if (threadIdx.x == 0) {
        out[0] = t0;
        out[1] = t1;
        out[2] = sqrt(t2);
    }
}

unsigned reduce_grid(uint64_t items) {
    uint64_t b = (items + kBlock * 8 - 1) / (kBlock * 8);
    if (b < 1) b = 1;
    if (b > unsigned(kReduceBlocks)) b = kReduceBlocks;
    return unsigned(b);
}

}  // namespace

hipError_t launch_probs_full(const void *amp, int dtype, int n, const int *perm_pos,
                             bool identity, double *out, hipStream_t s) {
    const uint64_t count = uint64_t(1) << n;
    uint64_t g = (count + kBlock * 4 - 1) / (kBlock * 4);
    if (g > 256u * 64u) g = 256u * 64u;
    const int tok = timer_begin("probs", s);
    if (identity) {
        if (dtype == QC_C64)
            hipLaunchKernelGGL((k_probs_full<float>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                               static_cast<const cx<float> *>(amp), count, out);
        else
            hipLaunchKernelGGL((k_probs_full<double>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                               static_cast<const cx<double> *>(amp), count, out);
    } else {
        PermArgs p{};
        p.m = n;
        for (int j = 0; j < n; ++j) p.src_pos[j] = uint32_t(perm_pos[j]);
        if (dtype == QC_C64)
            hipLaunchKernelGGL((k_probs_perm<float>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                               static_cast<const cx<float> *>(amp), count, p, out);
        else
            hipLaunchKernelGGL((k_probs_perm<double>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                               static_cast<const cx<double> *>(amp), count, p, out);
    }
    timer_end(tok, s);
    return hipGetLastError();
}

// Blocks per bin of the marginal kernel: enough blocks to fill the chip,
// at least 4096 indices per block.
static uint64_t marginal_chunks(int n, int m) {
    const uint64_t rest = uint64_t(1) << (n - m), bins = uint64_t(1) << m;
    uint64_t chunks = 1;
    while (bins * chunks < 4096 && rest / (chunks * 2) >= 4096) chunks *= 2;
    return chunks;
}

size_t probs_marginal_work(int n, int m) {
    const uint64_t chunks = marginal_chunks(n, m);
    return chunks == 1 ? 0 : size_t((uint64_t(1) << m) * chunks);
}

hipError_t launch_probs_marginal(const void *amp, int dtype, int n, int m, const int *pos,
                                 double *out, double *work, size_t work_elems, hipStream_t s) {
    MarginalArgs a{};
    a.m = m;
    for (int j = 0; j < m; ++j) a.bin_off[j] = uint64_t(1) << pos[j];
    int sorted[QC_MAX_QUBITS];
    for (int j = 0; j < m; ++j) sorted[j] = pos[j];
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) {
            const int t = sorted[j];
            sorted[j] = sorted[j - 1];
            sorted[j - 1] = t;
        }
    for (int j = 0; j < m; ++j) a.pos[j] = uint32_t(sorted[j]);
    a.rest = uint64_t(1) << (n - m);
    const uint64_t bins = uint64_t(1) << m;
    const uint64_t chunks = marginal_chunks(n, m);
    // one chunk per bin: every block writes its bin's sum straight into out
    // (no partials, so no workspace bound: a 24-qubit marginal has 2^24 bins)
    const bool direct = chunks == 1;
    if ((!direct && bins * chunks > work_elems) || bins * chunks > 0x7fffffffull)
        return hipErrorInvalidValue;
    double *dst = direct ? out : work;
    a.chunks = int(chunks);
    a.chunk = a.rest / chunks;
    a.items = bins * chunks;
    const unsigned grid = unsigned(a.items < (uint64_t(1) << 20) ? a.items : (uint64_t(1) << 20));
    // pairs of neighbouring amplitudes when bit 0 is not listed, every
    // chunk is even and the state is 16-byte aligned
    const bool pair = dtype == QC_C64 && a.pos[0] >= 1 && (a.chunk % 2) == 0 &&
                      (reinterpret_cast<uintptr_t>(amp) & 15) == 0;
    const int tok = timer_begin("probs_marginal", s);
    if (dtype == QC_C64 && pair)
        hipLaunchKernelGGL((k_probs_marginal<float, true>), dim3(grid),
                           dim3(kBlock), 0, s, static_cast<const cx<float> *>(amp), a, dst);
    else if (dtype == QC_C64)
        hipLaunchKernelGGL((k_probs_marginal<float, false>), dim3(grid),
                           dim3(kBlock), 0, s, static_cast<const cx<float> *>(amp), a, dst);
    else
        hipLaunchKernelGGL((k_probs_marginal<double, false>), dim3(grid),
                           dim3(kBlock), 0, s, static_cast<const cx<double> *>(amp), a, dst);
    if (!direct)
        hipLaunchKernelGGL(k_sum_rows, dim3(unsigned(bins)), dim3(kBlock), 0, s, work, int(bins),
                           int(chunks), out);
    timer_end(tok, s);
    return hipGetLastError();
}

template <typename R>
void launch_expect_nt(const cx<R> *amp, const ExpectArgs &a, double *work, unsigned grid,
                      hipStream_t s) {
    static_assert(kExpectMaxTerms == 32, "term-count buckets assume at most 32 terms");
    if (a.n_terms <= 1)
        hipLaunchKernelGGL((k_expect_group<R, 1>), dim3(grid), dim3(kBlock), 0, s, amp, a, work);
    else if (a.n_terms <= 4)
        hipLaunchKernelGGL((k_expect_group<R, 4>), dim3(grid), dim3(kBlock), 0, s, amp, a, work);
    else if (a.n_terms <= 8)
        hipLaunchKernelGGL((k_expect_group<R, 8>), dim3(grid), dim3(kBlock), 0, s, amp, a, work);
    else if (a.n_terms <= 16)
        hipLaunchKernelGGL((k_expect_group<R, 16>), dim3(grid), dim3(kBlock), 0, s, amp, a, work);
    else
        hipLaunchKernelGGL((k_expect_group<R, 32>), dim3(grid), dim3(kBlock), 0, s, amp, a, work);
}

hipError_t launch_expect_group(const void *amp, int dtype, int n, uint64_t xmask, int hpos,
                               int n_terms, const uint64_t *zmask, const int *phase,
                               double *term_vals, double *work, hipStream_t s) {
    if (n_terms < 1 || n_terms > kExpectMaxTerms) return hipErrorInvalidValue;
    ExpectArgs a{};
    a.xmask = xmask;
    a.hpos = hpos;
    a.n_terms = n_terms;
    a.n_items = hpos < 0 ? (uint64_t(1) << n) : (uint64_t(1) << (n - 1));
    for (int t = 0; t < n_terms; ++t) {
        a.zmask[t] = zmask[t];
        a.phase[t] = phase[t] & 3;
    }
    const unsigned grid = reduce_grid(a.n_items);
    const int tok = timer_begin("expect", s);
    if (dtype == QC_C64)
        launch_expect_nt<float>(static_cast<const cx<float> *>(amp), a, work, grid, s);
    else
        launch_expect_nt<double>(static_cast<const cx<double> *>(amp), a, work, grid, s);
    hipLaunchKernelGGL(k_sum_rows, dim3(unsigned(n_terms)), dim3(kBlock), 0, s, work, n_terms,
                       int(grid), term_vals);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_expect_combine(const double *term_vals, const double *coeff_dev, int n_terms,
                                 int per_term, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_expect_combine, dim3(1), dim3(64), 0, s, term_vals, coeff_dev, n_terms,
                       per_term, out);
    return hipGetLastError();
}

hipError_t launch_diff(const void *a, int dt_a, const void *b, int dt_b, uint64_t count,
                       double *out, double *work, hipStream_t s) {
    const unsigned grid = reduce_grid(count);
    const int tok = timer_begin("diff", s);
    if (dt_a == QC_C64 && dt_b == QC_C64)
        hipLaunchKernelGGL((k_diff<float, float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cx<float> *>(a), static_cast<const cx<float> *>(b), count, work);
    else if (dt_a == QC_C64 && dt_b == QC_C128)
        hipLaunchKernelGGL((k_diff<float, double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cx<float> *>(a), static_cast<const cx<double> *>(b), count, work);
    else if (dt_a == QC_C128 && dt_b == QC_C64)
        hipLaunchKernelGGL((k_diff<double, float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cx<double> *>(a), static_cast<const cx<float> *>(b), count, work);
    else
        hipLaunchKernelGGL((k_diff<double, double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<const cx<double> *>(a), static_cast<const cx<double> *>(b), count, work);
    hipLaunchKernelGGL(k_diff_final, dim3(1), dim3(kBlock), 0, s, work, int(grid), out);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
