// Measurement kernels for gfx950 (QCLAB section 3.3 and the examples of
// sections 5.1/5.2): collapse onto an outcome with renormalisation, the
// reduced state of the unmeasured qubits, and shot sampling by inverse CDF.
//
// Collapse: P(b) = sum of |psi_i|^2 over the indices whose measured qubit
// reads b (computed by the marginal-probability kernels, FP64), then
// psi_i <- psi_i / sqrt(P(b)) on those indices and 0 elsewhere.  The scale
// is read from device memory, so no host round trip is needed.
//
// Sampling: the caller supplies uniforms u in [0, 1); shot k returns the
// first index i whose cumulative weight (index order) exceeds u_k times the
// total weight (so unnormalised states sample their normalised law).
// The cumulative sum is two-level: FP64 sums of 4096-amplitude chunks, an
// exclusive scan over the chunk sums (one block, fixed order), then a
// sequential walk inside the selected chunk.
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

template <typename R>
__device__ inline double norm2(cx<R> a) {
    return double(a.re) * double(a.re) + double(a.im) * double(a.im);
}

// prob[0..1] = P(0), P(1) of bit p; keeps or zeroes and rescales
template <typename R>
__global__ __launch_bounds__(kBlock) void k_collapse(cx<R> *amp, uint64_t count, int p, int b,
                                                     const double *prob, double *prob_out) {
    const double P = prob[b];
    if (blockIdx.x == 0 && threadIdx.x == 0 && prob_out) prob_out[0] = P;
    if (!(P > 0.0)) return;                 // impossible outcome: state unchanged
    const R scale = R(1.0 / sqrt(P));
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        const bool keep = ((i >> p) & 1) == uint64_t(b);
        cx<R> v = amp[i];
        v.re = keep ? v.re * scale : R(0);
        v.im = keep ? v.im * scale : R(0);
        amp[i] = v;
    }
}

// Reset of bit p, branch b (section 3.3 resets): with P = prob[b], the
// pair (i0, i1 = i0 | 2^p) becomes (a_b / sqrt(P), 0): the outcome-b
// collapse followed, for b = 1, by X on the bit.  One pass over the pairs.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_reset(cx<R> *amp, uint64_t pairs, int p, int b,
                                                  const double *prob, double *prob_out) {
    const double P = prob[b];
    if (blockIdx.x == 0 && threadIdx.x == 0 && prob_out) prob_out[0] = P;
    if (!(P > 0.0)) return;                 // impossible outcome: state unchanged
    const R scale = R(1.0 / sqrt(P));
    const uint64_t bit = uint64_t(1) << p;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < pairs; g += stride) {
        const uint64_t i0 = insert_zero(g, p);
        const cx<R> v = amp[b ? (i0 | bit) : i0];
        amp[i0] = cx<R>{v.re * scale, v.im * scale};
        amp[i0 | bit] = cx<R>{R(0), R(0)};
    }
}

// Shot counts over m listed bits: counts[s] = number of shots whose index
// reads s at the listed positions (pos[0] = most significant bit of s).
// Integer atomics: the result does not depend on the order of the adds.
struct CountArgs {
    uint32_t pos[QC_MAX_QUBITS];
    int m;
};
__global__ __launch_bounds__(kBlock) void k_zero_i64(int64_t *p, uint64_t count) {
    const uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < count) p[i] = 0;
}
__global__ __launch_bounds__(kBlock) void k_count(const int64_t *idx, int shots, const CountArgs a,
                                                  unsigned long long *counts) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= shots) return;
    const uint64_t i = uint64_t(idx[k]);
    uint64_t s = 0;
    for (int j = 0; j < a.m; ++j) s = (s << 1) | ((i >> a.pos[j]) & 1);
    atomicAdd(counts + s, 1ull);
}

struct ReduceArgs {
    uint32_t pos[QC_MAX_QUBITS];  // ascending positions of the known qubits
    int m;
    uint64_t fixed;               // known values at their positions
    uint64_t count;               // 2^(n-m) output amplitudes
};

template <typename R>
__global__ __launch_bounds__(kBlock) void k_reduced(const cx<R> *src, cx<R> *dst,
                                                    const ReduceArgs a) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t r = uint64_t(blockIdx.x) * kBlock + threadIdx.x; r < a.count; r += stride)
        dst[r] = src[insert_zeros(r, a.pos, a.m) | a.fixed];
}

// Chunks of 2^cb amplitudes: cb = 12 for registers of 12..33 qubits, the
// whole register below that, and larger chunks above, so that there are at
// most 2^21 chunks (their sums and prefix sums live in the FP64 workspace).
constexpr int kChunkBits = 12;
constexpr int kMaxChunkLog = 21;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_chunk_sums(const cx<R> *amp, int cb, double *csum) {
    __shared__ double red[kWaves];
    const uint64_t base = uint64_t(blockIdx.x) << cb;
    double acc = 0.0;
    for (int j = threadIdx.x; j < (1 << cb); j += kBlock) acc += norm2(amp[base + j]);
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += red[w];
        csum[blockIdx.x] = t;
    }
}

// exclusive scan of csum[0..nc) into cpre[0..nc], cpre[nc] = total; one block
__global__ __launch_bounds__(1024) void k_scan(const double *csum, uint64_t nc, double *cpre) {
    __shared__ double seg[1024];
    const uint64_t per = (nc + 1023) / 1024;
    const uint64_t b0 = threadIdx.x * per, b1 = b0 + per < nc ? b0 + per : nc;
    double s = 0.0;
    for (uint64_t c = b0; c < b1; ++c) s += csum[c];
    seg[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < 1024; ++t) {
            const double v = seg[t];
            seg[t] = run;
            run += v;
        }
        cpre[nc] = run;
    }
    __syncthreads();
    double run = seg[threadIdx.x];
    for (uint64_t c = b0; c < b1; ++c) {
        cpre[c] = run;
        run += csum[c];
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_sample(const cx<R> *amp, const double *cpre,
                                                   uint64_t nc, int cb, const double *u,
                                                   int shots, int64_t *out) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= shots) return;
    // target cumulative weight; the distribution is normalised by its total
    const double total = cpre[nc];
    double x = u[k] * total;
    if (!(x < total)) x = total * (1.0 - 0x1p-52);
    // last chunk c with cpre[c] <= x (chunks with zero weight are skipped
    // because cpre[c + 1] == cpre[c] there)
    uint64_t lo = 0, hi = nc;   // invariant: cpre[lo] <= x or lo == 0
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (cpre[mid] <= x) lo = mid;
        else hi = mid;
    }
    const uint64_t base = lo << cb;
    double acc = cpre[lo];
    int64_t last_nonzero = -1;
    for (int j = 0; j < (1 << cb); ++j) {
        const double w = norm2(amp[base + j]);
        if (w > 0.0) last_nonzero = int64_t(base + j);
        acc += w;
        if (acc > x && w > 0.0) {
            out[k] = int64_t(base + j);
            return;
        }
    }
    // rounding left x beyond this chunk's sum: take its last non-zero index
    out[k] = last_nonzero >= 0 ? last_nonzero : int64_t(base);
}

unsigned grid_for(uint64_t items) {
    uint64_t g = (items + kBlock * 4 - 1) / (kBlock * 4);
    if (g < 1) g = 1;
    if (g > 256u * 64u) g = 256u * 64u;
    return unsigned(g);
}

}  // namespace

hipError_t launch_collapse(void *amp, int dtype, int n, int p, int b, const double *prob,
                           double *prob_out, hipStream_t s) {
    const uint64_t count = uint64_t(1) << n;
    const unsigned g = grid_for(count);
    const int tok = timer_begin("collapse", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_collapse<float>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(amp), count, p, b, prob, prob_out);
    else
        hipLaunchKernelGGL((k_collapse<double>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(amp), count, p, b, prob, prob_out);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_reset(void *amp, int dtype, int n, int p, int b, const double *prob,
                        double *prob_out, hipStream_t s) {
    const uint64_t pairs = uint64_t(1) << (n - 1);
    const unsigned g = grid_for(pairs);
    const int tok = timer_begin("reset", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_reset<float>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(amp), pairs, p, b, prob, prob_out);
    else
        hipLaunchKernelGGL((k_reset<double>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(amp), pairs, p, b, prob, prob_out);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_count(const int64_t *idx, int shots, int m, const int *pos, int64_t *counts,
                        hipStream_t s) {
    CountArgs a{};
    a.m = m;
    for (int j = 0; j < m; ++j) a.pos[j] = uint32_t(pos[j]);
    const uint64_t bins = uint64_t(1) << m;
    hipLaunchKernelGGL(k_zero_i64, dim3(unsigned((bins + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, counts, bins);
    if (shots > 0)
        hipLaunchKernelGGL(k_count, dim3(unsigned((shots + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, idx, shots, a, reinterpret_cast<unsigned long long *>(counts));
    return hipGetLastError();
}

hipError_t launch_reduced(const void *src, void *dst, int dtype, int n, int m, const int *pos,
                          const int *val, hipStream_t s) {
    ReduceArgs a{};
    int srt[QC_MAX_QUBITS];
    for (int j = 0; j < m; ++j) {
        srt[j] = pos[j];
        if (val[j]) a.fixed |= uint64_t(1) << pos[j];
    }
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0 && srt[j - 1] > srt[j]; --j) {
            const int t = srt[j];
            srt[j] = srt[j - 1];
            srt[j - 1] = t;
        }
    for (int j = 0; j < m; ++j) a.pos[j] = uint32_t(srt[j]);
    a.m = m;
    a.count = uint64_t(1) << (n - m);
    const unsigned g = grid_for(a.count);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_reduced<float>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cx<float> *>(src), static_cast<cx<float> *>(dst), a);
    else
        hipLaunchKernelGGL((k_reduced<double>), dim3(g), dim3(kBlock), 0, s,
                           static_cast<const cx<double> *>(src), static_cast<cx<double> *>(dst), a);
    return hipGetLastError();
}

hipError_t launch_sample(const void *amp, int dtype, int n, const double *u, int shots,
                         int64_t *out, double *work, size_t work_elems, hipStream_t s) {
    int cb = n - kMaxChunkLog > kChunkBits ? n - kMaxChunkLog : kChunkBits;
    if (cb > n) cb = n;
    const uint64_t nc = uint64_t(1) << (n - cb);
    if (2 * nc + 1 > work_elems || nc > 0x7fffffffull) return hipErrorInvalidValue;
    double *csum = work, *cpre = work + nc;
    const int tok = timer_begin("sample", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_chunk_sums<float>), dim3(unsigned(nc)), dim3(kBlock), 0, s,
                           static_cast<const cx<float> *>(amp), cb, csum);
    else
        hipLaunchKernelGGL((k_chunk_sums<double>), dim3(unsigned(nc)), dim3(kBlock), 0, s,
                           static_cast<const cx<double> *>(amp), cb, csum);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, csum, nc, cpre);
    const unsigned g = unsigned((shots + kBlock - 1) / kBlock);
    if (shots > 0) {
        if (dtype == QC_C64)
            hipLaunchKernelGGL((k_sample<float>), dim3(g), dim3(kBlock), 0, s,
                               static_cast<const cx<float> *>(amp), cpre, nc, cb, u, shots, out);
        else
            hipLaunchKernelGGL((k_sample<double>), dim3(g), dim3(kBlock), 0, s,
                               static_cast<const cx<double> *>(amp), cpre, nc, cb, u, shots, out);
    }
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
