// Pauli-string expectation values, many terms per pass over the state.
//
// For P = i^ny X^x Z^z (x, z bit masks, ny = number of Y factors),
//   <psi|P|psi> = sum_j Re[ i^ny (-1)^popc(j & z) conj(psi_{j^x}) psi_j ]
// (the single non-zero entry of each row of the Kronecker product of Pauli
// matrices, QCLAB section 5.2 for the one-qubit case).  When every bit of x
// is a tile bit, j and j ^ x lie in the same tile, so one pass that stages
// tiles in LDS serves every such term, and every diagonal term (x = 0), at
// once: a transverse-field Ising Hamiltonian on n qubits needs about
// (n - 6) / (m - 6) passes instead of one per X term.
//
// Per tile and term, each thread sums its share, the wavefront adds its 64
// lanes with shuffles, and lane 0 adds the result to the wavefront's slot in
// LDS; after the last tile the slots are added in wavefront order.  Tiles
// are visited in a fixed order for a fixed grid, so the sums are
// deterministic.
//
// Diagonal terms: thread t owns the elements i = t + kBlock k, k < K, so
// (-1)^popc(i & z) = (-1)^popc(t & z_lo) (-1)^popc(k & z_k) with z_lo, z_k
// the parts of z below and above bit kLoBits.  The thread takes |psi_i|^2
// once per tile and their K Walsh sums W[h] = sum_k (-1)^popc(k & h) w_k.
// The leading diagonal terms of a launch then take the transform further,
// over the six lane bits (butterflies between lanes), and each one reads
// its coefficient from the eight wavefronts (through LDS) with their signs:
// one thread per term, no reduction per term.  Diagonal terms after the
// first X term take one W entry and one sign and a wavefront sum.
#include "qc_tile_ops.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

using tile::kBlock;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxK = 8;   // elements per thread: tiles of at most kBlock x 8 = 2^12

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Bytes before the term slots: the tile, or the diagonal terms'
// coefficients (kBlock doubles per element a thread holds) if larger.
__host__ __device__ inline size_t diag_region(int T, size_t elem) {
    const size_t tile = size_t(T) * elem;
    const size_t co = size_t(T > kBlock ? T : kBlock) * sizeof(double);
    return tile > co ? tile : co;
}
static_assert(kWaves == 8, "frequency bits 6..8 are the wavefront index");

constexpr int kXReg = 12;   // terms per launch whose partial sums stay in registers

// This thread's share of <psi|P|psi> over the tile in LDS for term tm
// (without the sign of its Z bits outside the tile).  Diagonal terms take
// the per-thread Walsh sums W (see below) instead.
template <typename R>
__device__ inline double term_pairs(const cx<R> *lds, const ExpectTerm &tm, int half) {
    double acc = 0.0;
    const uint32_t hb = tm.xtop;
    if (tm.zc == 0 && tm.ph == 0) {   // uniform: X factors only, both signs +1
        for (int g = threadIdx.x; g < half; g += kBlock) {
            const uint32_t i = ((uint32_t(g) >> hb) << (hb + 1)) | (uint32_t(g) & ((1u << hb) - 1));
            const uint32_t ix = i ^ tm.xc;
            const double ar = double(lds[i].re), ai = double(lds[i].im);
            const double br = double(lds[ix].re), bi = double(lds[ix].im);
            acc += br * ar + bi * ai;
        }
        return 2.0 * acc;
    }
    for (int g = threadIdx.x; g < half; g += kBlock) {
        const uint32_t i = ((uint32_t(g) >> hb) << (hb + 1)) | (uint32_t(g) & ((1u << hb) - 1));
        const uint32_t ix = i ^ tm.xc;
        const double ar = double(lds[i].re), ai = double(lds[i].im);
        const double br = double(lds[ix].re), bi = double(lds[ix].im);
        const double c1 = br * ar + bi * ai;
        const double c2 = br * ai - bi * ar;
        const double si = (__popc(i & tm.zc) & 1) ? -1.0 : 1.0;
        const double sx = (__popc(ix & tm.zc) & 1) ? -1.0 : 1.0;
        switch (tm.ph) {
        case 0: acc += (si + sx) * c1; break;
        case 1: acc -= (si - sx) * c2; break;
        case 2: acc -= (si + sx) * c1; break;
        default: acc += (si - sx) * c2; break;
        }
    }
    return acc;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_expect_tiles(const cx<R> *amp, const TileArgs a,
                                                         const ExpectTerm *terms, int nt,
                                                         double *part) {
    extern __shared__ unsigned char smem[];
    const int T = 1 << a.m;
    const int K = T > kBlock ? T >> tile::kLoBits : 1;   // elements per thread
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    double *coef = reinterpret_cast<double *>(smem);   // reuses the tile (see diag_region)
    double *wacc = reinterpret_cast<double *>(smem + diag_region(T, sizeof(cx<R>)));   // [term][wave]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < nt * kWaves; i += kBlock) wacc[i] = 0.0;
    // the leading diagonal terms (thread d keeps the sum of term d)
    int nd = 0;
    while (nd < nt && nd < kBlock && terms[nd].xc == 0) ++nd;
    double dacc = 0.0;
    double xacc[kXReg];
#pragma unroll
    for (int j = 0; j < kXReg; ++j) xacc[j] = 0.0;
    const uint64_t off_lo =
        tile::deposit(uint32_t(threadIdx.x) & (T - 1), a.pos, a.m < tile::kLoBits ? a.m : tile::kLoBits);
    const uint64_t mask = tile::hi_mask(a.pos, a.m);
    const int half = T >> 1;
    for (uint64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const uint64_t base = insert_zeros(t, a.pos, a.m);
        tile::tile_load<R>(lds, amp, base, off_lo, mask, T);
        __syncthreads();
        double W[kMaxK];
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
            const int i = int(threadIdx.x) + k * kBlock;
            W[k] = 0.0;
            if (k < K && i < T) {
                const double re = double(lds[i].re), im = double(lds[i].im);
                W[k] = re * re + im * im;
            }
        }
#pragma unroll
        for (int h = 1; h < kMaxK; h <<= 1)
#pragma unroll
            for (int k = 0; k < kMaxK; ++k)
                if (!(k & h)) {
                    const double u = W[k], v = W[k | h];
                    W[k] = u + v;
                    W[k | h] = u - v;
                }
        // the first kXReg terms after the leading diagonal ones keep their
        // per-thread sums in registers across tiles (one reduction per
        // launch); further terms are reduced per tile
#pragma unroll
        for (int j = 0; j < kXReg; ++j) {
            const int k = nd + j;
            if (k >= nt) break;   // uniform
            const ExpectTerm tm = terms[k];
            double v;
            if (tm.xc == 0) {   // a diagonal term after an X term: its Walsh sum
                const uint32_t zk = tm.zc >> tile::kLoBits;   // uniform, < K
                double w = W[0];
#pragma unroll
                for (int h = 1; h < kMaxK; ++h)
                    if (zk == uint32_t(h)) w = W[h];
                v = (__popc(threadIdx.x & tm.zc) & 1) ? -w : w;
            } else {
                v = term_pairs<R>(lds, tm, half);
            }
            // the Z bits outside the tile give every amplitude of it one sign
            xacc[j] += (__popcll(base & terms[k].z_hi) & 1) ? -v : v;
        }
        for (int k = nd + kXReg; k < nt; ++k) {
            const ExpectTerm tm = terms[k];
            double acc = 0.0;
            if (tm.xc == 0) {
                const uint32_t zk = tm.zc >> tile::kLoBits;   // uniform, < K
                double w = W[0];
#pragma unroll
                for (int h = 1; h < kMaxK; ++h)
                    if (zk == uint32_t(h)) w = W[h];
                acc = (__popc(threadIdx.x & tm.zc) & 1) ? -w : w;
            } else if (tm.zc == 0 && tm.ph == 0) {   // uniform: X factors only
                // both signs +1: the pair gives 2 Re(conj(b) a)
                const uint32_t hb = tm.xtop;
                for (int g = threadIdx.x; g < half; g += kBlock) {
                    const uint32_t i = ((uint32_t(g) >> hb) << (hb + 1)) | (uint32_t(g) & ((1u << hb) - 1));
                    const uint32_t ix = i ^ tm.xc;
                    const double ar = double(lds[i].re), ai = double(lds[i].im);
                    const double br = double(lds[ix].re), bi = double(lds[ix].im);
                    acc += br * ar + bi * ai;
                }
                acc *= 2.0;
            } else {
                // pairs (i, i ^ xc), i with a zero at the top bit of xc
                const uint32_t hb = tm.xtop;
                for (int g = threadIdx.x; g < half; g += kBlock) {
                    const uint32_t i = ((uint32_t(g) >> hb) << (hb + 1)) | (uint32_t(g) & ((1u << hb) - 1));
                    const uint32_t ix = i ^ tm.xc;
                    const double ar = double(lds[i].re), ai = double(lds[i].im);
                    const double br = double(lds[ix].re), bi = double(lds[ix].im);
                    // conj(b) a = c1 + i c2
                    const double c1 = br * ar + bi * ai;
                    const double c2 = br * ai - bi * ar;
                    const double si = (__popc(i & tm.zc) & 1) ? -1.0 : 1.0;
                    const double sx = (__popc(ix & tm.zc) & 1) ? -1.0 : 1.0;
                    // Re[i^ny (si conj(b) a + sx conj(a) b)]
                    switch (tm.ph) {
                    case 0: acc += (si + sx) * c1; break;
                    case 1: acc -= (si - sx) * c2; break;
                    case 2: acc -= (si + sx) * c1; break;
                    default: acc += (si - sx) * c2; break;
                    }
                }
            }
            acc = wave_sum(acc);
            // the Z bits outside the tile give every amplitude of it one sign
            if (__popcll(base & tm.z_hi) & 1) acc = -acc;
            if (lane == 0) wacc[k * kWaves + wave] += acc;
        }
        if (nd > 0) {   // uniform
            // the Walsh transform of |psi|^2 continued over the six lane
            // bits: W[h] of lane l becomes the coefficient of frequency
            // (l, h) summed over this wavefront's elements
#pragma unroll
            for (int b = 0; b < 6; ++b)
#pragma unroll
                for (int h = 0; h < kMaxK; ++h) {
                    const double p = __shfl_xor(W[h], 1 << b, 64);
                    W[h] = ((lane >> b) & 1) ? p - W[h] : W[h] + p;
                }
            __syncthreads();   // every read of the tile is done: its LDS now holds the coefficients
            for (int h = 0; h < K; ++h) coef[h * kBlock + int(threadIdx.x)] = W[h];
            __syncthreads();
            // term d: frequency zc = (wavefront bits, lane bits, h); the
            // eight wavefronts' coefficients combine with their signs
            if (int(threadIdx.x) < nd) {
                const ExpectTerm tm = terms[threadIdx.x];
                const uint32_t lu = tm.zc & 63u, wu = (tm.zc >> 6) & 7u, hu = tm.zc >> tile::kLoBits;
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) {
                    const double c = coef[hu * kBlock + uint32_t(w) * 64 + lu];
                    v += (__popc(uint32_t(w) & wu) & 1) ? -c : c;
                }
                // the Z bits outside the tile give every amplitude of it one sign
                dacc += (__popcll(base & tm.z_hi) & 1) ? -v : v;
            }
        }
        __syncthreads();
    }
    // the register-held sums: one wavefront reduction per term per launch
#pragma unroll
    for (int j = 0; j < kXReg; ++j) {
        if (nd + j >= nt) break;   // uniform
        const double v = wave_sum(xacc[j]);
        if (lane == 0) wacc[(nd + j) * kWaves + wave] += v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nt; k += kBlock) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += wacc[k * kWaves + w];
        part[size_t(k) * gridDim.x + blockIdx.x] = k < nd ? dacc : s;   // thread k < nd owns term k
    }
}

// vals[k] = sum over the blocks of part[k][.], in block order
__global__ __launch_bounds__(kBlock) void k_expect_rows(const double *part, int cols,
                                                        double *vals) {
    __shared__ double red[kWaves];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < cols; c += kBlock) acc += part[size_t(k) * cols + c];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kWaves; ++w) s += red[w];
        vals[k] = s;
    }
}

}  // namespace

unsigned expect_tiles_grid(uint64_t n_tiles) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint64_t g = uint64_t(cus) * 2;
    if (g > n_tiles) g = n_tiles;
    return unsigned(g < 1 ? 1 : g);
}

hipError_t launch_expect_tiles(const void *amp, int dtype, const TileArgs &a,
                               const ExpectTerm *terms_dev, int nt, double *vals, double *part,
                               hipStream_t s) {
    if (nt < 1 || nt > kExpectTileMaxTerms || a.m < 1 || (1 << a.m) > kBlock * kMaxK)
        return hipErrorInvalidValue;
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t lds = diag_region(1 << a.m, elem) + size_t(nt) * kWaves * sizeof(double);
    if (lds > 65536) return hipErrorInvalidValue;
    const unsigned grid = expect_tiles_grid(a.n_tiles);
    const int tok = timer_begin("expect_tiles", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_expect_tiles<float>), dim3(grid), dim3(kBlock), lds, s,
                           static_cast<const cx<float> *>(amp), a, terms_dev, nt, part);
    else
        hipLaunchKernelGGL((k_expect_tiles<double>), dim3(grid), dim3(kBlock), lds, s,
                           static_cast<const cx<double> *>(amp), a, terms_dev, nt, part);
    hipLaunchKernelGGL(k_expect_rows, dim3(unsigned(nt)), dim3(kBlock), 0, s, part, int(grid), vals);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
