// Adjoint-method gradient kernels (Jones & Gacon, arXiv:2009.02823; the
// QCLAB paper itself has no gradients).
//
// For E(theta) = <phi|H|phi>, phi = U_L ... U_1 psi and a parametrised gate
// U_k = exp(-i theta G / 2) with G in {X, Y, Z}:
//   dE/dtheta_k = 2 Re <lam_k| dU_k/dtheta |phi_{k-1}> = Im <lam_k| G |phi_k>,
// where phi_k is the state after gate k and lam_k = U_{k+1}^+ .. U_L^+ H phi.
//
// The backward sweep runs the reversed, adjoint gate list on BOTH vectors
// in LDS tile runs: a tile of phi and the matching tile of lam are loaded
// together, and for every rotation of the run the FP64 partial
// Im <lam|G|phi> over the tile is taken right before its inverse is applied
// to both tiles.  A run of G gates costs 4 state-sizes of HBM traffic in
// total instead of 4 per gate.  Partials are kept per (rotation,
// workgroup) and summed in a fixed order afterwards.
#include "qc_rt_ops.h"
#include "qc_tile_ops.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

constexpr int kBlock = tile::kBlock;
constexpr int kWaves = kBlock / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// lam = H psi = sum_t c_t i^ny (-1)^popc((j^x) & z) psi_{j^x}  (ACC: lam +=)
template <typename R, bool ACC>
__global__ __launch_bounds__(kBlock) void k_pauli_apply(const cx<R> *psi, cx<R> *out,
                                                        uint64_t count,
                                                        const PauliTermDev *terms, int nt) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < count; j += stride) {
        const cx<R> pj = psi[j];
        double ar = 0.0, ai = 0.0;
        if (ACC) {
            ar = double(out[j].re);
            ai = double(out[j].im);
        }
        for (int t = 0; t < nt; ++t) {
            const PauliTermDev T = terms[t];
            const uint64_t k = j ^ T.x;
            const cx<R> a = T.x ? psi[k] : pj;
            const double s = (__popcll(k & T.z) & 1) ? -T.c : T.c;
            double vr = s * double(a.re), vi = s * double(a.im);
            switch (T.ph) {
            case 0: break;
            case 1: { const double tr = -vi; vi = vr; vr = tr; } break;
            case 2: vr = -vr; vi = -vi; break;
            default: { const double tr = vi; vi = -vr; vr = tr; } break;
            }
            ar += vr;
            ai += vi;
        }
        out[j] = cx<R>{R(ar), R(ai)};
    }
}

// Im <lam|G|phi> over one pair (i0, i1 = i0 with bit b set) for generator
// G (1 = X, 2 = Y, 3 = Z), in the state's precision; the caller accumulates
// in FP64.  conj(a) b = (ar br + ai bi) + i (ar bi - ai br).
template <typename R>
__device__ inline R grad_pair(cx<R> f0, cx<R> f1, cx<R> l0, cx<R> l1, int gen) {
    if (gen == 3) return (l0.re * f0.im - l0.im * f0.re) - (l1.re * f1.im - l1.im * f1.re);
    if (gen == 1) return (l0.re * f1.im - l0.im * f1.re) + (l1.re * f0.im - l1.im * f0.re);
    return -(l0.re * f1.re + l0.im * f1.im) + (l1.re * f0.re + l1.im * f0.im);
}

// The one-qubit matrix u = [u0 u1; u2 u3] on the pair (a0, a1): general
// complex, real (imaginary parts zero) or diagonal.
enum { APPLY_NONE = 0, APPLY_GENERAL = 1, APPLY_REAL = 2, APPLY_DIAG = 3 };
template <typename R, int A>
__device__ inline void apply_pair(cx<R> &a0, cx<R> &a1, cx<R> u0, cx<R> u1, cx<R> u2, cx<R> u3) {
    if (A == APPLY_GENERAL) {
        const cx<R> z{R(0), R(0)};
        const cx<R> b0 = cfma(u1, a1, cfma(u0, a0, z));
        a1 = cfma(u3, a1, cfma(u2, a0, z));
        a0 = b0;
    } else if (A == APPLY_REAL) {
        const cx<R> b0{u0.re * a0.re + u1.re * a1.re, u0.re * a0.im + u1.re * a1.im};
        a1 = cx<R>{u2.re * a0.re + u3.re * a1.re, u2.re * a0.im + u3.re * a1.im};
        a0 = b0;
    } else if (A == APPLY_DIAG) {
        a0 = cmul(u0, a0);
        a1 = cmul(u3, a1);
    }
}

// Im <lam|G|phi> over the pairs of compressed bit b of one tile (partial of
// this thread).  Unless A == APPLY_NONE, the one-qubit matrix u on bit b is
// then applied to both tiles in the same pass (the partial uses the values
// before the update).  tile::kItems independent pairs per thread per step.
template <typename R, int A>
__device__ inline double grad_pairs(cx<R> *f, cx<R> *l, int m, int b, int gen, const double *u) {
    cx<R> u0{}, u1{}, u2{}, u3{};
    if (A != APPLY_NONE) {
        u0 = tile::ld_u<R>(u, 0);
        u1 = tile::ld_u<R>(u, 1);
        u2 = tile::ld_u<R>(u, 2);
        u3 = tile::ld_u<R>(u, 3);
    }
    const int npairs = 1 << (m - 1);
    const uint32_t bit = 1u << b;
    double acc = 0.0;
    for (int g0 = threadIdx.x; g0 < npairs; g0 += kBlock * tile::kItems) {
        uint32_t i0[tile::kItems];
        bool ok[tile::kItems];
        cx<R> f0[tile::kItems], f1[tile::kItems], l0[tile::kItems], l1[tile::kItems];
#pragma unroll
        for (int k = 0; k < tile::kItems; ++k) {
            const int g = g0 + k * kBlock;
            ok[k] = g < npairs;
            i0[k] = tile::ins0(uint32_t(g), b);
            if (ok[k]) {
                f0[k] = f[i0[k]];
                f1[k] = f[i0[k] | bit];
                l0[k] = l[i0[k]];
                l1[k] = l[i0[k] | bit];
            }
        }
#pragma unroll
        for (int k = 0; k < tile::kItems; ++k) {
            if (!ok[k]) continue;
            acc += double(grad_pair<R>(f0[k], f1[k], l0[k], l1[k], gen));
            if (A != APPLY_NONE) {
                apply_pair<R, A>(f0[k], f1[k], u0, u1, u2, u3);
                apply_pair<R, A>(l0[k], l1[k], u0, u1, u2, u3);
                f[i0[k]] = f0[k];
                f[i0[k] | bit] = f1[k];
                l[i0[k]] = l0[k];
                l[i0[k] | bit] = l1[k];
            }
        }
    }
    return acc;
}

// TILE_GRAD_APPLY2: two gradient-and-apply steps on bit b in one pass over
// the pairs: partial 1 (generator gen1), matrix u on both tiles, partial 2
// (generator gen2) on the updated values, matrix w on both tiles.
template <typename R, int A1, int A2>
__device__ inline void grad_pairs2(cx<R> *f, cx<R> *l, int m, int b, int gen1, int gen2,
                                   const double *u, const double *w, double &acc1, double &acc2) {
    const cx<R> u0 = tile::ld_u<R>(u, 0), u1 = tile::ld_u<R>(u, 1), u2 = tile::ld_u<R>(u, 2),
                u3 = tile::ld_u<R>(u, 3);
    const cx<R> w0 = tile::ld_u<R>(w, 0), w1 = tile::ld_u<R>(w, 1), w2 = tile::ld_u<R>(w, 2),
                w3 = tile::ld_u<R>(w, 3);
    // complex128: two pairs per thread per step (four would pass 128 registers)
    constexpr int kI = sizeof(R) == sizeof(float) ? tile::kItems : 2;
    const int npairs = 1 << (m - 1);
    const uint32_t bit = 1u << b;
    acc1 = 0.0;
    acc2 = 0.0;
    for (int g0 = threadIdx.x; g0 < npairs; g0 += kBlock * kI) {
        uint32_t i0[kI];
        bool ok[kI];
        cx<R> f0[kI], f1[kI], l0[kI], l1[kI];
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            const int g = g0 + k * kBlock;
            ok[k] = g < npairs;
            i0[k] = tile::ins0(uint32_t(g), b);
            if (ok[k]) {
                f0[k] = f[i0[k]];
                f1[k] = f[i0[k] | bit];
                l0[k] = l[i0[k]];
                l1[k] = l[i0[k] | bit];
            }
        }
#pragma unroll
        for (int k = 0; k < kI; ++k) {
            if (!ok[k]) continue;
            acc1 += double(grad_pair<R>(f0[k], f1[k], l0[k], l1[k], gen1));
            apply_pair<R, A1>(f0[k], f1[k], u0, u1, u2, u3);
            apply_pair<R, A1>(l0[k], l1[k], u0, u1, u2, u3);
            acc2 += double(grad_pair<R>(f0[k], f1[k], l0[k], l1[k], gen2));
            apply_pair<R, A2>(f0[k], f1[k], w0, w1, w2, w3);
            apply_pair<R, A2>(l0[k], l1[k], w0, w1, w2, w3);
            f[i0[k]] = f0[k];
            f[i0[k] | bit] = f1[k];
            l[i0[k]] = l0[k];
            l[i0[k] | bit] = l1[k];
        }
    }
}

// At most 128 VGPRs (4 wavefronts per SIMD): two workgroups per CU, which
// their LDS (two tiles of at most 32 KiB) allows.
template <typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_adjoint_tiles(cx<R> *phi, cx<R> *lam, const TileArgs a,
                                                          const TileOp *ops,
                                                          const int32_t *slot_row, int n_slots,
                                                          double *partial, int cols) {
    extern __shared__ unsigned char smem[];
    __shared__ double acc[kAdjointMaxSlots];
    // per-wavefront partials of a gradient op, double-buffered: thread 0
    // adds them into acc at the start of the next op, after the op's own
    // closing barrier, so a gradient costs no barrier of its own (the
    // additions keep their order: one slot at a time, wavefronts in order)
    // (a paired op leaves a second partial in red2 for slot pend_slot2)
    __shared__ double red[2][kWaves], red2[2][kWaves];
    int pend_slot = -1, pend_slot2 = -1, pend_buf = 0;
    auto fold = [&]() {
        if (pend_slot >= 0 && threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += red[pend_buf][w];
            acc[pend_slot] += s;
            if (pend_slot2 >= 0) {
                s = 0.0;
                for (int w = 0; w < kWaves; ++w) s += red2[pend_buf][w];
                acc[pend_slot2] += s;
            }
        }
        pend_slot = -1;
        pend_slot2 = -1;
    };
    __shared__ TileOp op_slot[2];
    __shared__ tile::PhaseTables<R> pt;
    const int T = 1 << a.m;
    cx<R> *lp = reinterpret_cast<cx<R> *>(smem);
    cx<R> *ll = lp + T;
    for (int s = threadIdx.x; s < n_slots; s += kBlock) acc[s] = 0.0;
    __syncthreads();
    const uint64_t off_lo =
        tile::deposit(uint32_t(threadIdx.x) & (T - 1), a.pos, a.m < tile::kLoBits ? a.m : tile::kLoBits);
    const uint64_t mask = tile::hi_mask(a.pos, a.m);
    for (uint64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const uint64_t base = insert_zeros(t, a.pos, a.m);
        tile::tile_load<R>(lp, phi, base, off_lo, mask, T);
        tile::tile_load<R>(ll, lam, base, off_lo, mask, T);
        // ops are staged through LDS as in tile::apply_ops
        if (a.n_ops > 0) tile::stage_now(&op_slot[0], &ops[0]);
        __syncthreads();
        for (int o = 0; o < a.n_ops; ++o) {
            const TileOp &op = op_slot[o & 1];
            const bool next = o + 1 < a.n_ops;
            tile::OpStage st;
            if (next) tile::stage_fetch(st, &ops[o + 1]);
            fold();
            if ((base & op.cmask_hi) == op.cval_hi) {   // uniform per tile
                if (op.kind == TILE_GRAD || op.kind == TILE_GRAD_APPLY ||
                    op.kind == TILE_GRAD_APPLY_REAL || op.kind == TILE_GRAD_APPLY_DIAG) {
                    double v;
                    switch (op.kind) {   // uniform
                    case TILE_GRAD: v = grad_pairs<R, APPLY_NONE>(lp, ll, a.m, op.b0, op.b1, nullptr); break;
                    case TILE_GRAD_APPLY_REAL: v = grad_pairs<R, APPLY_REAL>(lp, ll, a.m, op.b0, op.b1, op.u); break;
                    case TILE_GRAD_APPLY_DIAG: v = grad_pairs<R, APPLY_DIAG>(lp, ll, a.m, op.b0, op.b1, op.u); break;
                    default: v = grad_pairs<R, APPLY_GENERAL>(lp, ll, a.m, op.b0, op.b1, op.u); break;
                    }
                    v = wave_sum(v);
                    if ((threadIdx.x & 63) == 0) red[o & 1][threadIdx.x >> 6] = v;
                    pend_slot = op.pad;
                    pend_buf = o & 1;
                } else if (op.kind == TILE_GRAD_APPLY2_DIAG_REAL) {
                    double v1, v2;
                    const int gens = op.b1;
                    grad_pairs2<R, APPLY_DIAG, APPLY_REAL>(lp, ll, a.m, op.b0, gens & 15, gens >> 4,
                                                           op.u, op.u1, v1, v2);
                    v1 = wave_sum(v1);
                    v2 = wave_sum(v2);
                    if ((threadIdx.x & 63) == 0) {
                        red[o & 1][threadIdx.x >> 6] = v1;
                        red2[o & 1][threadIdx.x >> 6] = v2;
                    }
                    pend_slot = op.pad & 0xffff;
                    pend_slot2 = op.pad >> 16;
                    pend_buf = o & 1;
                } else if (op.kind == TILE_PHASES) {
                    const bool any = tile::phases_table<R>(pt.tab, pt.hix, a.m, base, op, op.b0,
                                                           uint32_t(op.b1));   // uniform
                    __syncthreads();
                    if (any) {
                        tile::phases_apply<R>(lp, a.m, pt.tab, pt.hix, uint32_t(op.b1));
                        tile::phases_apply<R>(ll, a.m, pt.tab, pt.hix, uint32_t(op.b1));
                    }
                } else {
                    // the backward op lists hold no TILE_KRON (built with kron_max 1)
                    tile::apply_one<R, false>(lp, a.m, op);
                    tile::apply_one<R, false>(ll, a.m, op);
                }
            }
            if (next) tile::stage_store(st, &op_slot[(o + 1) & 1]);
            __syncthreads();
        }
        fold();
        tile::tile_store<R>(phi, lp, base, off_lo, mask, T);
        tile::tile_store<R>(lam, ll, base, off_lo, mask, T);
        __syncthreads();
    }
    for (int s = threadIdx.x; s < n_slots; s += kBlock)
        partial[size_t(slot_row[s]) * cols + blockIdx.x] = acc[s];
}

// Backward pass on register tiles: a tile of phi and the matching tile of
// lam live in registers under one layout; gradient ops take their partial
// before applying the inverse rotation to both, every other op is applied
// to each vector in turn (exchanges through LDS one vector at a time).
// Partials: one column per wavefront in LDS, folded in wavefront order at
// the end, one value per (gradient slot, workgroup).
template <typename R, int RB>
__global__ __launch_bounds__(rt::kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_rt_adjoint(cx<R> *__restrict__ phi, cx<R> *__restrict__ lam, const RtArgs a,
                  const RtOp *__restrict__ ops, const unsigned char *__restrict__ tabs,
                  const int32_t *slot_row, int n_slots, double *partial, int cols) {
    constexpr int E = 1 << RB;
    extern __shared__ unsigned char smem[];
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    const size_t xbytes = (size_t(1) << a.m) * sizeof(cx<R>);
    double *gacc = reinterpret_cast<double *>(smem + xbytes);              // [slot][wave]
    unsigned char *ltab = smem + xbytes + size_t(kRtAdjSlots) * 8 * sizeof(double);
    const uint32_t tid = threadIdx.x;
    const bool act = tid < (1u << a.tb);
    for (uint32_t i = tid; i < uint32_t(n_slots) * 8; i += blockDim.x) gacc[i] = 0.0;
    for (uint32_t i = tid; i < a.lds_tab_bytes / 16; i += blockDim.x)
        reinterpret_cast<uint4 *>(ltab)[i] = reinterpret_cast<const uint4 *>(tabs)[i];
    __syncthreads();
    const rt::Tabs tb{ltab, tabs, tid & 63u,
                      uint32_t(__builtin_amdgcn_readfirstlane(int(tid >> 6)))};
    uint64_t thr_ld = 0, thr_st = 0;
    for (int k = 0; k < a.tb; ++k) {
        const uint64_t bit = (tid >> k) & 1u;
        thr_ld |= bit << a.ld_thr[k];
        thr_st |= bit << a.st_thr[k];
    }
    for (uint64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const uint64_t base = insert_zeros(t, a.pos, a.m);
        cx<R> vp[E], vl[E];
        if (act) {
            const cx<R> *sp = phi + base + thr_ld, *sl = lam + base + thr_ld;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint64_t off = rt::reg_offset<RB>(e, a.ld_reg);
                vp[e] = sp[off];
                vl[e] = sl[off];
            }
        }
        rt::run_ops2<R, RB>(vp, vl, lds, gacc, base, tid, act, ops, a.n_ops, tb);
        if (act) {
            cx<R> *dp = phi + base + thr_st, *dl = lam + base + thr_st;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint64_t off = rt::reg_offset<RB>(e, a.st_reg);
                dp[off] = vp[e];
                dl[off] = vl[e];
            }
        }
    }
    __syncthreads();
    for (int sl = int(tid); sl < n_slots; sl += int(blockDim.x)) {
        double v = 0.0;
        for (int w = 0; w < 8; ++w) v += gacc[sl * 8 + w];
        partial[size_t(slot_row[sl]) * cols + blockIdx.x] = v;
    }
}

// g_op[i] = sum of row i of the partials (fixed order), then
// grad[p] = sum over the rotations of parameter p (CSR, op order).
__global__ __launch_bounds__(kBlock) void k_grad_rows(const double *partial, int cols,
                                                      double *g_op) {
    __shared__ double lds[kWaves];
    const int row = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < cols; c += kBlock) acc += partial[size_t(row) * cols + c];
    double v = wave_sum(acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kWaves; ++w) r += lds[w];
        g_op[row] = r;
    }
}

__global__ void k_grad_scatter(const double *g_op, const int *ptr, const int *idx, int n_params,
                               double *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    double s = 0.0;
    for (int k = ptr[p]; k < ptr[p + 1]; ++k) s += g_op[idx[k]];
    grad[p] = s;
}

}  // namespace

unsigned adjoint_tile_grid(uint64_t n_tiles) {
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint64_t cap = uint64_t(cus) * 4;
    return unsigned(n_tiles < cap ? n_tiles : cap);
}

hipError_t launch_pauli_apply(const void *psi, void *out, int dtype, int n,
                              const PauliTermDev *terms, int nt, bool accumulate, hipStream_t s) {
    const uint64_t count = uint64_t(1) << n;
    uint64_t g = (count + kBlock * 4 - 1) / (kBlock * 4);
    if (g > 256u * 64u) g = 256u * 64u;
    const int tok = timer_begin("pauli_apply", s);
#define QC_PA_LAUNCH(R, A)                                                                       \
    hipLaunchKernelGGL((k_pauli_apply<R, A>), dim3(unsigned(g)), dim3(kBlock), 0, s,             \
                       static_cast<const cx<R> *>(psi), static_cast<cx<R> *>(out), count, terms, nt)
    if (dtype == QC_C64) {
        if (accumulate) QC_PA_LAUNCH(float, true); else QC_PA_LAUNCH(float, false);
    } else {
        if (accumulate) QC_PA_LAUNCH(double, true); else QC_PA_LAUNCH(double, false);
    }
#undef QC_PA_LAUNCH
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_adjoint_tiles(void *phi, void *lam, int dtype, const TileArgs &a,
                                const TileOp *ops_dev, const int32_t *slot_row_dev, int n_slots,
                                double *partial, unsigned cols, hipStream_t s) {
    if (n_slots > kAdjointMaxSlots) return hipErrorInvalidValue;
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t lds = 2 * (size_t(1) << a.m) * elem;
    if (lds > 65536) return hipErrorInvalidValue;
    const int tok = timer_begin(dtype == QC_C64 ? "adjoint_tiles_c64" : "adjoint_tiles_c128", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_adjoint_tiles<float>), dim3(cols), dim3(kBlock), lds, s,
                           static_cast<cx<float> *>(phi), static_cast<cx<float> *>(lam), a, ops_dev,
                           slot_row_dev, n_slots, partial, int(cols));
    else
        hipLaunchKernelGGL((k_adjoint_tiles<double>), dim3(cols), dim3(kBlock), lds, s,
                           static_cast<cx<double> *>(phi), static_cast<cx<double> *>(lam), a,
                           ops_dev, slot_row_dev, n_slots, partial, int(cols));
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_rt_adjoint(void *phi, void *lam, int dtype, const RtArgs &a, const RtOp *ops_dev,
                             const unsigned char *tabs_dev, const int32_t *slot_row_dev,
                             int n_slots, double *partial, unsigned cols, hipStream_t s) {
    const int rb = rt_adj_reg_bits(dtype);
    if (n_slots < 0 || n_slots > kRtAdjSlots || a.m < rb || a.m > rb + kRtMaxTB ||
        a.tb != a.m - rb || a.lds_tab_bytes % 16)
        return hipErrorInvalidValue;
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t lds = (size_t(1) << a.m) * elem + size_t(kRtAdjSlots) * 8 * sizeof(double) +
                       a.lds_tab_bytes;
    if (lds > 80 * 1024) return hipErrorInvalidValue;
    const unsigned threads = 1u << (a.tb < 6 ? 6 : a.tb);
    const int tok = timer_begin(dtype == QC_C64 ? "rt_adjoint_c64" : "rt_adjoint_c128", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_rt_adjoint<float, 3>), dim3(cols), dim3(threads), lds, s,
                           static_cast<cx<float> *>(phi), static_cast<cx<float> *>(lam), a, ops_dev,
                           tabs_dev, slot_row_dev, n_slots, partial, int(cols));
    else
        hipLaunchKernelGGL((k_rt_adjoint<double, 2>), dim3(cols), dim3(threads), lds, s,
                           static_cast<cx<double> *>(phi), static_cast<cx<double> *>(lam), a,
                           ops_dev, tabs_dev, slot_row_dev, n_slots, partial, int(cols));
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(const double *partial, int rows, int cols, double *g_op,
                                const int *ptr, const int *idx, int n_params, double *grad,
                                hipStream_t s) {
    if (rows > 0)
        hipLaunchKernelGGL(k_grad_rows, dim3(unsigned(rows)), dim3(kBlock), 0, s, partial, cols,
                           g_op);
    if (n_params > 0)
        hipLaunchKernelGGL(k_grad_scatter, dim3(unsigned((n_params + 255) / 256)), dim3(256), 0,
                           s, g_op, ptr, idx, n_params, grad);
    return hipGetLastError();
}

}  // namespace qcx
