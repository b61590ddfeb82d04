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
#include "qc_lanes.h"
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

// ---- register tiles: one wavefront per tile ----------------------------------
//
// Lane l holds the 16 amplitudes e of its tile in registers, in the state's
// precision, and converts them to FP64 once; every product and sum is FP64.
// For a term whose X bits lie in the tile, the partner of element (l, e) is
// element (l ^ xl, e ^ xr).  The kernel takes the terms whose X bits are
// one element bit (a register of the lane itself, compile-time index per
// bit; each pair taken once and doubled), one lane bit below 4 (the partner
// through a DPP row shift; the lane with the bit clear takes the pair twice)
// or any lane mask (an LDS permute; each lane counts its own side).  The
// host gives each X term a kind that names its case.  Complex64 passes
// also write the tile to a padded LDS buffer and read it back under a
// second layout in which the lane bits of some terms are element bits; the
// host assigns those terms to the second layout.  The sign of the Z bits
// outside the tile and on the lane bits is applied per tile and lane, and
// each lane adds its term partials to its own LDS slots.
//
// Diagonal terms: see k_expect_reg.
//
// The next tile's loads are issued before the current tile is evaluated.
// Tiles are dealt to wavefronts round-robin for a fixed grid, and every
// sum runs in a fixed order: the result is deterministic.
constexpr int kRegE = 1 << kExpRegB;
constexpr int kRegBlock = 256;
constexpr int kRegWaves = kRegBlock / 64;
static_assert(kRegE == 16, "the element switches below cover 16 elements");

// streaming load of one amplitude (read once: non-temporal)
template <typename R>
__device__ __forceinline__ cx<R> load_stream(const cx<R> *p) {
    typedef R r2 __attribute__((ext_vector_type(2)));
    const r2 v = __builtin_nontemporal_load(reinterpret_cast<const r2 *>(p));
    return cx<R>{v.x, v.y};
}

// Re[conj(b) a] (ODD false) or Im[conj(b) a] (ODD true) in FP64
template <typename R, bool ODD>
__device__ __forceinline__ double pair_prod(cx<R> a, cx<R> b) {
    const double ar = double(a.re), ai = double(a.im), br = double(b.re), bi = double(b.im);
    return ODD ? fma(br, ai, -bi * ar) : fma(br, ar, bi * ai);
}

// -1.0 when bit e of the uniform mask is set, else +1.0 (a scalar value)
__device__ __forceinline__ double elem_sign(uint32_t zsign, int e) {
    return ((zsign >> e) & 1u) ? -1.0 : 1.0;
}

// Sum over the lane's elements of a term whose X bits are the element mask
// XR != 0 (no lane bits): the member with the lowest bit of XR clear.
template <typename R, int XR, bool ODD>
__device__ __forceinline__ double elem_pairs(const cx<R> *v, uint32_t zsign) {
    constexpr int lowb = XR & -XR;
    double acc = 0.0;
    if (!ODD && zsign == 0) {   // uniform: no element signs
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            if (e & lowb) continue;
            const cx<R> a = v[e], b = v[e ^ XR];
            acc = fma(double(b.re), double(a.re), acc);
            acc = fma(double(b.im), double(a.im), acc);
        }
    } else {
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            if (e & lowb) continue;
            acc = fma(elem_sign(zsign, e), pair_prod<R, ODD>(v[e], v[e ^ XR]), acc);
        }
    }
    return 2.0 * acc;
}

// amplitude of lane (lane ^ m) (m uniform)
__device__ __forceinline__ cx<float> shfl_amp(cx<float> x, uint32_t m) {
    return cx<float>{__shfl_xor(x.re, int(m), 64), __shfl_xor(x.im, int(m), 64)};
}
__device__ __forceinline__ cx<double> shfl_amp(cx<double> x, uint32_t m) {
    return cx<double>{__shfl_xor(x.re, int(m), 64), __shfl_xor(x.im, int(m), 64)};
}

// Sum over the lane's elements of a term whose X bits are the lane mask xl
// (any mask: the partner comes from an LDS permute; every lane counts its
// own side of each pair)
template <typename R, bool ODD>
__device__ __forceinline__ double lane_term(const cx<R> *v, uint32_t xl, uint32_t zsign) {
    double acc = 0.0;
    if (!ODD && zsign == 0) {   // uniform: no element signs
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const cx<R> a = v[e], b = shfl_amp(v[e], xl);
            acc = fma(double(b.re), double(a.re), acc);
            acc = fma(double(b.im), double(a.im), acc);
            if (e % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound the shuffles in flight
        }
    } else {
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            acc = fma(elem_sign(zsign, e), pair_prod<R, ODD>(v[e], shfl_amp(v[e], xl)), acc);
            if (e % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound the shuffles in flight
        }
    }
    return acc;
}

// A term whose X bits are the one lane bit B < 4: the lanes with bit B
// clear fetch their partner's amplitudes through a DPP row shift (VALU, no
// LDS) and count each pair twice; the lanes with bit B set count nothing.
template <int B, bool ODD>
__device__ __forceinline__ double lane_bit_term(const cx<double> *w, uint32_t zsign, uint32_t lane) {
    double acc = 0.0;
    if (!ODD && zsign == 0) {   // uniform: no element signs
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            acc = fma(lanes::up<B>(w[e].re), w[e].re, acc);
            acc = fma(lanes::up<B>(w[e].im), w[e].im, acc);
            if (e % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound the partners held at once
        }
    } else {
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const cx<double> b{lanes::up<B>(w[e].re), lanes::up<B>(w[e].im)};
            acc = fma(elem_sign(zsign, e), pair_prod<double, ODD>(w[e], b), acc);
            if (e % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound the partners held at once
        }
    }
    return ((lane >> B) & 1u) ? 0.0 : 2.0 * acc;
}

// Register-tile pass.  Diagonal terms, with p_e = |psi|^2 of element e:
//  - z_hi = 0 (every Z bit in the tile): the lane adds p_e over its tiles
//    (pacc); after the last tile, sum_e (-1)^popc(e & zr) pacc_e with the
//    sign of the lane bits, over the wavefront;
//  - z_hi != 0: the sign outside the tile changes from tile to tile.  For
//    each distinct pair (zsign, zl) of the launch the wavefront forms the
//    tile's sum sum_{l,e} (-1)^popc(l & zl) (-1)^popc(e & zr) p_{l,e} and
//    parks it on lane k for the k-th tile of a group of 64; after 64 tiles
//    each term takes the signs of its z_hi over the 64 tile bases at once
//    (one lane each) and one wavefront sum.
// X terms: one lane-local sum per tile and term, added to the lane's slot
// in LDS with the signs outside the element bits.
template <typename R, bool DIAG>
__global__ __launch_bounds__(kRegBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_expect_reg(const cx<R> *__restrict__ amp, const ExpRegArgs a,
                                                          const ExpRegTerm *__restrict__ terms,
                                                          double *__restrict__ part) {
    __shared__ double red[kRegWaves][kExpRegMaxX + kExpRegMaxD];
    extern __shared__ double dyn_lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = uint32_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)));
    const uint64_t nw = uint64_t(gridDim.x) * kRegWaves;
    uint64_t lane_off = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if ((lane >> k) & 1u) lane_off |= uint64_t(1) << a.lpos[k];
    uint64_t reg_off[kRegE];
#pragma unroll
    for (int e = 0; e < kRegE; ++e) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < kExpRegB; ++i)
            if ((e >> i) & 1) o |= uint64_t(1) << a.rpos[i];
        reg_off[e] = o;
    }
    const int nx = a.n_x, nxa = a.n_x - a.n_xb;
    double *wlds = dyn_lds + size_t(wave) * (expect_reg_wave_lds(a, sizeof(cx<R>)) / sizeof(double));
    // per-lane sums of the X terms across tiles (one slot per lane)
    double *xacc = wlds + lane;
    for (int k = 0; k < nx; ++k) xacc[64 * k] = 0.0;
    // lane k of rc: a pair's sum over the k-th tile of the current group
    double *rc = wlds + 64 * nx + lane;
    // transposition buffer: tile index j at j + tpad (j >> tsh); this lane's
    // slot offsets for the loaded layout (index lane + 64 e) and for the
    // transposed one (lane bits on tile bits tl, element bits on te); the
    // bits of the two parts are disjoint, so their padded offsets add
    constexpr bool kTrans = sizeof(R) == 4;   // complex64 only (LDS budget)
    auto padded = [&](uint32_t j) { return j + a.tpad * (j >> a.tsh); };
    uint32_t tr_lane = 0;
    for (int k = 0; k < 6; ++k)
        if ((lane >> k) & 1u) tr_lane |= 1u << a.tl[k];
    tr_lane = padded(tr_lane);
    const uint32_t wr_lane = padded(lane);
    cx<R> *tb = reinterpret_cast<cx<R> *>(wlds + 64 * (nx + a.n_c));
    if (DIAG) {
        for (int d = int(lane); d < a.n_d; d += 64) red[wave][kExpRegMaxX + d] = 0.0;
        for (int c = 0; c < a.n_c; ++c) rc[64 * c] = 0.0;
    }
    double pacc[kRegE];
#pragma unroll
    for (int e = 0; e < kRegE; ++e) pacc[e] = 0.0;
    // this tile's lane in rc, and the first tile of the group there
    uint32_t slot = 0;
    uint64_t t_grp = 0;

    // tiles in flight per wavefront, each in its own registers (two tiles
    // of complex64 measured no faster than one)
    constexpr int PF = 1;
    cx<R> buf[PF][kRegE];
    uint64_t bbase[PF];
    uint64_t t = uint64_t(blockIdx.x) * kRegWaves + wave;
    auto issue = [&](cx<R> *dst, uint64_t &b, uint64_t tt) {
        if (tt < a.n_tiles) {
            b = insert_zeros(tt, a.pos, 6 + kExpRegB);
            const cx<R> *src = amp + b + lane_off;
#pragma unroll
            for (int e = 0; e < kRegE; ++e) dst[e] = load_stream<R>(src + reg_off[e]);
        }
    };
#pragma unroll
    for (int p = 0; p < PF; ++p) issue(buf[p], bbase[p], t + uint64_t(p) * nw);
    t_grp = t;
    // one tile: the tile in buffer `cur`, whose registers then take the
    // loads of the tile PF steps ahead
    auto one_tile = [&](cx<R> *cur, uint64_t &cbase) {
        const uint64_t base = cbase;
        if (kTrans && a.n_xb > 0) {   // uniform: the tile into the transposition buffer
#pragma unroll
            for (int e = 0; e < kRegE; ++e) tb[wr_lane + padded(64u * uint32_t(e))] = cur[e];
        }
        // the tile in FP64, converted once
        cx<double> w[kRegE];
#pragma unroll
        for (int e = 0; e < kRegE; ++e) w[e] = cx<double>{double(cur[e].re), double(cur[e].im)};
        issue(cur, cbase, t + uint64_t(PF) * nw);
        // X terms [k0, k1) on the tile w
        auto x_terms = [&](int k0, int k1) {
            for (int k = k0; k < k1; ++k) {   // uniform
                const ExpRegTerm tm = terms[k];
                // an empty asm that claims to change w: the pair products of
                // every element mask would otherwise be hoisted out of the term
                // loop (64 FP64 values held across it, spilled registers)
    #pragma unroll
                for (int e = 0; e < kRegE; ++e) asm volatile("" : "+v"(w[e].re), "+v"(w[e].im));
                double s = 0.0;
                switch (tm.kind) {   // uniform, one dispatch per term
                case 0: s = elem_pairs<double, 1, false>(w, tm.zsign); break;
                case 1: s = elem_pairs<double, 1, true>(w, tm.zsign); break;
                case 2: s = elem_pairs<double, 2, false>(w, tm.zsign); break;
                case 3: s = elem_pairs<double, 2, true>(w, tm.zsign); break;
                case 4: s = elem_pairs<double, 4, false>(w, tm.zsign); break;
                case 5: s = elem_pairs<double, 4, true>(w, tm.zsign); break;
                case 6: s = elem_pairs<double, 8, false>(w, tm.zsign); break;
                case 7: s = elem_pairs<double, 8, true>(w, tm.zsign); break;
                case 8: s = lane_bit_term<0, false>(w, tm.zsign, lane); break;
                case 9: s = lane_bit_term<0, true>(w, tm.zsign, lane); break;
                case 10: s = lane_bit_term<1, false>(w, tm.zsign, lane); break;
                case 11: s = lane_bit_term<1, true>(w, tm.zsign, lane); break;
                case 12: s = lane_bit_term<2, false>(w, tm.zsign, lane); break;
                case 13: s = lane_bit_term<2, true>(w, tm.zsign, lane); break;
                case 14: s = lane_bit_term<3, false>(w, tm.zsign, lane); break;
                case 15: s = lane_bit_term<3, true>(w, tm.zsign, lane); break;
                case 16: s = lane_term<double, false>(w, tm.xl, tm.zsign); break;
                case 17: s = lane_term<double, true>(w, tm.xl, tm.zsign); break;
                default: break;   // the host emits no other kinds
                }
                // Re[i^ph c]: ph 0 -> Re c, 1 -> -Im c, 2 -> -Re c, 3 -> Im c; then
                // the signs of the Z bits on the lane and outside the tile
                const uint32_t neg = uint32_t((tm.ph == 1 || tm.ph == 2) + __popc(lane & tm.zl) +
                                              __popcll(base & tm.z_hi)) & 1u;
                // LDS add without return: no wait on the slot's old value
                __hip_atomic_fetch_add(xacc + 64 * k, neg ? -s : s, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        };
        x_terms(0, nxa);
        if (DIAG) {
            double p[kRegE];
#pragma unroll
            for (int e = 0; e < kRegE; ++e) p[e] = fma(w[e].re, w[e].re, w[e].im * w[e].im);
            if (a.n_din > 0) {   // uniform
#pragma unroll
                for (int e = 0; e < kRegE; ++e) pacc[e] += p[e];
            }
            if (a.n_c > 0) {   // uniform
                double q[kExpRegMaxC];
#pragma unroll
                for (int c = 0; c < kExpRegMaxC; ++c) {
                    q[c] = 0.0;
                    if (c < a.n_c) {   // uniform
                        double s = 0.0;
#pragma unroll
                        for (int e = 0; e < kRegE; ++e) s = fma(elem_sign(a.csign[c], e), p[e], s);
                        q[c] = (__popc(lane & a.clane[c]) & 1) ? -s : s;
                    }
                }
#pragma unroll
                for (int c = 0; c < kExpRegMaxC; ++c)
                    if (c < a.n_c) {   // uniform: every lane takes part in the sum
                        const double qs = lanes::wave_sum(q[c]);
                        if (lane == slot) rc[64 * c] = qs;
                    }
            }
            ++slot;
            if (slot == 64 || t + nw >= a.n_tiles) {   // uniform: the group's terms
                if (a.n_c > 0) {
                    const uint64_t bl = insert_zeros(t_grp + uint64_t(lane) * nw, a.pos, 6 + kExpRegB);
                    for (int d = 0; d < a.n_d; ++d) {   // uniform
                        const ExpRegTerm dt = terms[nx + d];
                        if (dt.ck < 0) continue;
                        double r = rc[64 * dt.ck];
                        r = lane < slot ? ((__popcll(bl & dt.z_hi) & 1) ? -r : r) : 0.0;
                        r = lanes::wave_sum(r);
                        if (lane == 0) red[wave][kExpRegMaxX + d] += r;
                    }
                }
                slot = 0;
                t_grp = t + nw;
            }
        }
        if (kTrans && a.n_xb > 0) {   // uniform: the transposed tile
            // LDS accesses of one wavefront are performed in order: the
            // fences only keep the compiler from moving them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int f = 0; f < kRegE; ++f) {
                uint32_t o = 0;
#pragma unroll
                for (int i = 0; i < kExpRegB; ++i)
                    if ((f >> i) & 1) o |= 1u << a.te[i];
                const cx<R> x = tb[tr_lane + padded(o)];
                w[f] = cx<double>{double(x.re), double(x.im)};
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            x_terms(nxa, nx);
        }
    };
    while (t < a.n_tiles) {   // uniform
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            if (t >= a.n_tiles) break;
            one_tile(buf[p], bbase[p]);
            t += nw;
        }
    }
    // per-wavefront sums, then the block's partial per term in wavefront order
    for (int k = 0; k < nx; ++k) {   // uniform
        const double s = lanes::wave_sum(xacc[64 * k]);
        if (lane == 0) red[wave][k] = s;
    }
    if (DIAG && a.n_din > 0) {
        for (int d = 0; d < a.n_d; ++d) {   // uniform
            const ExpRegTerm dt = terms[nx + d];
            if (dt.ck >= 0) continue;
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < kRegE; ++e) s = fma(elem_sign(dt.zsign, e), pacc[e], s);
            s = lanes::wave_sum((__popc(lane & dt.zl) & 1) ? -s : s);
            if (lane == 0) red[wave][kExpRegMaxX + d] = s;
        }
    }
    __syncthreads();
    const int nt = nx + (DIAG ? a.n_d : 0);
    for (int k = threadIdx.x; k < nt; k += kRegBlock) {
        const int col = k < nx ? k : kExpRegMaxX + (k - nx);
        double s = 0.0;
#pragma unroll
        for (int wv = 0; wv < kRegWaves; ++wv) s += red[wv][col];
        part[size_t(k) * gridDim.x + blockIdx.x] = s;
    }
}

// ---- lam = H psi on register tiles -------------------------------------------
//
// (P psi)_j = i^ph (-1)^popc((j ^ x) & z) psi_{j ^ x}: every amplitude of the
// output takes, for each term of the pass, its partner's amplitude (from
// another lane by a shuffle, or from a register of the lane) times
// c i^ph and the sign of the partner's index.  Diagonal terms: per lane
// A_h = sum of c (-1)^popc((base | lane) & z) over the terms of element mask
// h, then element e takes sum_h A_h (-1)^popc(e & h).  Products and sums in
// FP64, one rounding per amplitude and launch.  The first launch writes
// lam; the later ones (ACC) add to it.

// L += q * i^PH * b
template <int PH>
__device__ __forceinline__ void add_phase(double &lr, double &li, double q, double br, double bi) {
    if (PH == 0) { lr = fma(q, br, lr); li = fma(q, bi, li); }
    if (PH == 1) { lr = fma(-q, bi, lr); li = fma(q, br, li); }
    if (PH == 2) { lr = fma(-q, br, lr); li = fma(-q, bi, li); }
    if (PH == 3) { lr = fma(q, bi, lr); li = fma(-q, br, li); }
}

// a term whose X bits are the lane mask xl: the partner of (l, e) is (l ^ xl, e)
template <int PH>
__device__ __forceinline__ void pauli_lane(double *lr, double *li, const cx<double> *w, uint32_t xl,
                                           uint32_t zsign, double p) {
#pragma unroll
    for (int e = 0; e < kRegE; ++e) {
        const double br = __shfl_xor(w[e].re, int(xl), 64), bi = __shfl_xor(w[e].im, int(xl), 64);
        add_phase<PH>(lr[e], li[e], ((zsign >> e) & 1u) ? -p : p, br, bi);
        if (e % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound the shuffles in flight
    }
}

// a term whose X bit is element bit XR: the partner of (l, e) is (l, e ^ XR)
template <int PH, int XR>
__device__ __forceinline__ void pauli_elem(double *lr, double *li, const cx<double> *w, uint32_t zsign,
                                           double p) {
#pragma unroll
    for (int e = 0; e < kRegE; ++e)
        add_phase<PH>(lr[e], li[e], ((zsign >> (e ^ XR)) & 1u) ? -p : p, w[e ^ XR].re, w[e ^ XR].im);
}

template <int PH>
__device__ __forceinline__ void pauli_term(double *lr, double *li, const cx<double> *w,
                                           const ExpRegTerm &tm, double p) {
    switch (tm.xr) {
    case 0: pauli_lane<PH>(lr, li, w, tm.xl, tm.zsign, p); break;
    case 1: pauli_elem<PH, 1>(lr, li, w, tm.zsign, p); break;
    case 2: pauli_elem<PH, 2>(lr, li, w, tm.zsign, p); break;
    case 4: pauli_elem<PH, 4>(lr, li, w, tm.zsign, p); break;
    case 8: pauli_elem<PH, 8>(lr, li, w, tm.zsign, p); break;
    default: break;   // the host gives no other masks
    }
}

template <typename R, bool DIAG, bool ACC>
__global__ __launch_bounds__(kRegBlock) void k_pauli_reg(const cx<R> *__restrict__ psi,
                                                         cx<R> *__restrict__ lam, const ExpRegArgs a,
                                                         const ExpRegTerm *__restrict__ terms,
                                                         const double *__restrict__ coef) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = uint32_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)));
    const uint64_t nw = uint64_t(gridDim.x) * kRegWaves;
    uint64_t lane_off = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        if ((lane >> k) & 1u) lane_off |= uint64_t(1) << a.lpos[k];
    uint64_t reg_off[kRegE];
#pragma unroll
    for (int e = 0; e < kRegE; ++e) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < kExpRegB; ++i)
            if ((e >> i) & 1) o |= uint64_t(1) << a.rpos[i];
        reg_off[e] = o;
    }
    const int nx = a.n_x;
    for (uint64_t t = uint64_t(blockIdx.x) * kRegWaves + wave; t < a.n_tiles; t += nw) {
        const uint64_t base = insert_zeros(t, a.pos, 6 + kExpRegB);
        const cx<R> *src = psi + base + lane_off;
        cx<R> *dst = lam + base + lane_off;
        cx<double> w[kRegE];
        double lr[kRegE], li[kRegE];
#pragma unroll
        for (int e = 0; e < kRegE; ++e) {
            const cx<R> x = load_stream<R>(src + reg_off[e]);
            w[e] = cx<double>{double(x.re), double(x.im)};
            if (ACC) {
                const cx<R> y = dst[reg_off[e]];
                lr[e] = double(y.re);
                li[e] = double(y.im);
            } else {
                lr[e] = 0.0;
                li[e] = 0.0;
            }
        }
        for (int k = 0; k < nx; ++k) {   // uniform
            const ExpRegTerm tm = terms[k];
            // the partner's sign outside the element bits: its lane is lane ^ xl
            const uint32_t odd = uint32_t(__popc((lane ^ tm.xl) & tm.zl) + __popcll(base & tm.z_hi)) & 1u;
            const double p = odd ? -coef[k] : coef[k];
            switch (tm.ph) {
            case 0: pauli_term<0>(lr, li, w, tm, p); break;
            case 1: pauli_term<1>(lr, li, w, tm, p); break;
            case 2: pauli_term<2>(lr, li, w, tm, p); break;
            default: pauli_term<3>(lr, li, w, tm, p); break;
            }
        }
        if (DIAG) {
            double dg[kRegE];
#pragma unroll
            for (int e = 0; e < kRegE; ++e) dg[e] = 0.0;
            for (int h = 0; h < a.n_h; ++h) {   // uniform
                double A = 0.0;
                for (uint32_t d = a.hoff[h]; d < a.hoff[h + 1]; ++d) {   // uniform
                    const ExpRegTerm tm = terms[nx + int(d)];
                    const uint32_t odd = uint32_t(__popc(lane & tm.zl) + __popcll(base & tm.z_hi)) & 1u;
                    A += odd ? -coef[nx + int(d)] : coef[nx + int(d)];
                }
                const uint32_t hv = a.hval[h];
#pragma unroll
                for (int e = 0; e < kRegE; ++e)
                    dg[e] = (__popc(uint32_t(e) & hv) & 1) ? dg[e] - A : dg[e] + A;
            }
#pragma unroll
            for (int e = 0; e < kRegE; ++e) {
                lr[e] = fma(dg[e], w[e].re, lr[e]);
                li[e] = fma(dg[e], w[e].im, li[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < kRegE; ++e) dst[reg_off[e]] = cx<R>{R(lr[e]), R(li[e])};
    }
}

}  // namespace

unsigned expect_reg_grid(uint64_t n_tiles) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint64_t g = uint64_t(cus) * 2;
    const uint64_t need = (n_tiles + kRegWaves - 1) / kRegWaves;
    if (g > need) g = need;
    return unsigned(g < 1 ? 1 : g);
}

hipError_t launch_expect_reg(const void *amp, int dtype, const ExpRegArgs &a,
                             const ExpRegTerm *terms_dev, double *vals, double *part,
                             hipStream_t s) {
    const int nt = a.n_x + a.n_d;
    if (a.n_x < 0 || a.n_x > kExpRegMaxX || a.n_d < 0 || a.n_d > kExpRegMaxD || nt < 1 ||
        a.n_h < 0 || a.n_h > kExpRegMaxH || (a.n_d > 0 && a.n_h < 1) || a.n_tiles < 1 ||
        a.n_c < 0 || a.n_c > kExpRegMaxC || a.n_din < 0 || a.n_din > a.n_d)
        return hipErrorInvalidValue;
    if (a.n_xb < 0 || a.n_xb > a.n_x || (a.n_xb > 0 && (dtype != QC_C64 || a.tsh < 4 || a.tsh > 6)))
        return hipErrorInvalidValue;
    const unsigned grid = expect_reg_grid(a.n_tiles);
    const bool diag = a.n_d > 0;
    const size_t lds = kRegWaves * expect_reg_wave_lds(a, dtype == QC_C64 ? 8 : 16);
    const int tok = timer_begin("expect_reg", s);
    if (dtype == QC_C64) {
        if (diag)
            hipLaunchKernelGGL((k_expect_reg<float, true>), dim3(grid), dim3(kRegBlock), lds, s,
                               static_cast<const cx<float> *>(amp), a, terms_dev, part);
        else
            hipLaunchKernelGGL((k_expect_reg<float, false>), dim3(grid), dim3(kRegBlock), lds, s,
                               static_cast<const cx<float> *>(amp), a, terms_dev, part);
    } else {
        if (diag)
            hipLaunchKernelGGL((k_expect_reg<double, true>), dim3(grid), dim3(kRegBlock), lds, s,
                               static_cast<const cx<double> *>(amp), a, terms_dev, part);
        else
            hipLaunchKernelGGL((k_expect_reg<double, false>), dim3(grid), dim3(kRegBlock), lds, s,
                               static_cast<const cx<double> *>(amp), a, terms_dev, part);
    }
    hipLaunchKernelGGL(k_expect_rows, dim3(unsigned(nt)), dim3(kBlock), 0, s, part, int(grid), vals);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_pauli_reg(const void *psi, void *lam, int dtype, const ExpRegArgs &a,
                            const ExpRegTerm *terms_dev, const double *coef_dev, bool accumulate,
                            hipStream_t s) {
    const int nt = a.n_x + a.n_d;
    if (a.n_x < 0 || a.n_x > kExpRegMaxX || a.n_d < 0 || a.n_d > kExpRegMaxD || nt < 1 ||
        a.n_h < 0 || a.n_h > kExpRegMaxH || (a.n_d > 0 && a.n_h < 1) || a.n_tiles < 1)
        return hipErrorInvalidValue;
    const unsigned grid = expect_reg_grid(a.n_tiles);
    const bool diag = a.n_d > 0;
    const int tok = timer_begin("pauli_reg", s);
#define QC_PAULI_LAUNCH(R, D, A)                                                               \
    hipLaunchKernelGGL((k_pauli_reg<R, D, A>), dim3(grid), dim3(kRegBlock), 0, s,               \
                       static_cast<const cx<R> *>(psi), static_cast<cx<R> *>(lam), a, terms_dev, \
                       coef_dev)
    if (dtype == QC_C64) {
        if (diag) { if (accumulate) QC_PAULI_LAUNCH(float, true, true); else QC_PAULI_LAUNCH(float, true, false); }
        else { if (accumulate) QC_PAULI_LAUNCH(float, false, true); else QC_PAULI_LAUNCH(float, false, false); }
    } else {
        if (diag) { if (accumulate) QC_PAULI_LAUNCH(double, true, true); else QC_PAULI_LAUNCH(double, true, false); }
        else { if (accumulate) QC_PAULI_LAUNCH(double, false, true); else QC_PAULI_LAUNCH(double, false, false); }
    }
#undef QC_PAULI_LAUNCH
    timer_end(tok, s);
    return hipGetLastError();
}

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
