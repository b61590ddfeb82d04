// Gate-application kernels for gfx950: basis-state init, precision copy,
// K-target gates with arbitrary controls (K = 0, 1, 2), and the dense
// k-qubit block on the vector units.
//
// Gate application is the map psi -> (I_l (x) U' (x) I_r) psi of QCLAB
// section 3.2, evaluated without forming the register operator: every
// work item owns one "group" of 2^K amplitudes that differ only in the
// target bits (with the control bits pinned to their control values),
// loads them, multiplies by U' and stores them back in place.  Groups are
// disjoint, so no two lanes touch the same amplitude and no synchronisation
// is needed.  Consecutive lanes own consecutive groups: when the lowest
// pinned bit is high, each of the 2^K loads of a wave is one contiguous
// stream; when it is low, the 2^K loads of a wave still cover whole cache
// lines between them.
#include "qc_internal.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

constexpr int kBlock = 256;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_init_basis(cx<R> *amp, uint64_t count,
                                                       uint64_t basis) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        cx<R> v;
        v.re = (i == basis) ? R(1) : R(0);
        v.im = R(0);
        amp[i] = v;
    }
}

template <typename RD, typename RS>
__global__ __launch_bounds__(kBlock) void k_copy(cx<RD> *dst, const cx<RS> *src,
                                                 uint64_t count) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
        const cx<RS> v = src[i];
        dst[i] = cx<RD>{RD(v.re), RD(v.im)};
    }
}

// Same-precision copy in 16-byte units: each workgroup moves chunks of
// kBlock * 4 units (16 KiB), loads first; the grid normally holds one chunk
// per workgroup, which streams HBM best on MI355X.
typedef float floatx4_t __attribute__((ext_vector_type(4)));
constexpr int kCopyUnits = 4;
__global__ __launch_bounds__(kBlock) void k_copy_vec(floatx4_t *__restrict__ dst,
                                                     const floatx4_t *__restrict__ src,
                                                     uint64_t units) {
    const uint64_t chunk = uint64_t(kBlock) * kCopyUnits;
    for (uint64_t c = blockIdx.x; c * chunk < units; c += gridDim.x) {
        const uint64_t b = c * chunk + threadIdx.x;
        floatx4_t v[kCopyUnits];
#pragma unroll
        for (int u = 0; u < kCopyUnits; ++u)
            if (b + u * kBlock < units) v[u] = __builtin_nontemporal_load(src + b + u * kBlock);
#pragma unroll
        for (int u = 0; u < kCopyUnits; ++u)
            if (b + u * kBlock < units) __builtin_nontemporal_store(v[u], dst + b + u * kBlock);
    }
}

template <typename R, int K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_small_gate(const SmallGateArgs<R, K> a) {
    constexpr int D = 1 << K;
    const uint64_t g0 = uint64_t(blockIdx.x) * (kBlock * ITEMS) + threadIdx.x;
    cx<R> v[ITEMS][D];
    uint64_t base[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint64_t g = g0 + uint64_t(it) * kBlock;
        base[it] = insert_zeros(g, a.pos, a.n_pos) | a.or_bits;
        if (g < a.n_groups) {
#pragma unroll
            for (int r = 0; r < D; ++r) v[it][r] = a.amp[base[it] + a.tgt_off[r]];
        }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint64_t g = g0 + uint64_t(it) * kBlock;
        if (g >= a.n_groups) continue;
#pragma unroll
        for (int r = 0; r < D; ++r) {
            cx<R> acc{R(0), R(0)};
#pragma unroll
            for (int c = 0; c < D; ++c) acc = cfma(a.u[r * D + c], v[it][c], acc);
            a.amp[base[it] + a.tgt_off[r]] = acc;
        }
    }
}

// Dense k-qubit block on the vector units: one work item per column (one
// assignment of the non-target bits).  U lives in LDS; a multiplexed block
// holds 2^n_sel matrices and each column picks the one named by its
// selector bits.
template <typename R, int K>
__global__ __launch_bounds__(kBlock) void k_fused_valu(cx<R> *amp, uint64_t n_cols,
                                                       const FusedGeom g, const cx<R> *u_dev) {
    constexpr int D = 1 << K;
    extern __shared__ unsigned char smem_u[];
    cx<R> *U = reinterpret_cast<cx<R> *>(smem_u);
    const int n_mat = 1 << g.n_sel;
    for (int i = threadIdx.x; i < n_mat * D * D; i += kBlock) U[i] = u_dev[i];
    __syncthreads();
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t col = uint64_t(blockIdx.x) * kBlock + threadIdx.x; col < n_cols;
         col += stride) {
        const uint64_t base = insert_zeros(col, g.pos, g.n_pos);
        int sel = 0;
        for (int j = 0; j < g.n_sel; ++j) sel = (sel << 1) | int((base >> g.sel_pos[j]) & 1);
        const cx<R> *Us = U + sel * (D * D);
        cx<R> v[D];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] = amp[base + g.tgt_off[c]];
#pragma unroll 4
        for (int r = 0; r < D; ++r) {
            cx<R> acc{R(0), R(0)};
#pragma unroll
            for (int c = 0; c < D; ++c) acc = cfma(Us[r * D + c], v[c], acc);
            amp[base + g.tgt_off[r]] = acc;
        }
    }
}

inline unsigned grid_for(uint64_t items, uint64_t per_block, unsigned cap) {
    uint64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return unsigned(b);
}

constexpr unsigned kStreamGridCap = 256u * 64u;  // grid-stride kernels

template <typename R, int K>
hipError_t small_gate_typed(void *amp, int n, const int *tpos, int n_ctrl, const int *cpos,
                            const int *cval, const double *u, hipStream_t s) {
    SmallGateArgs<R, K> a{};
    a.amp = static_cast<cx<R> *>(amp);
    const int nfix = K + n_ctrl;
    a.n_groups = uint64_t(1) << (n - nfix);
    // sorted positions of all pinned bits
    int all[kMaxPos];
    for (int j = 0; j < K; ++j) all[j] = tpos[j];
    for (int j = 0; j < n_ctrl; ++j) all[K + j] = cpos[j];
    for (int i = 1; i < nfix; ++i)
        for (int j = i; j > 0 && all[j - 1] > all[j]; --j) {
            const int t = all[j];
            all[j] = all[j - 1];
            all[j - 1] = t;
        }
    for (int j = 0; j < nfix; ++j) a.pos[j] = uint32_t(all[j]);
    a.n_pos = nfix;
    a.or_bits = 0;
    for (int j = 0; j < n_ctrl; ++j)
        if (cval[j]) a.or_bits |= uint64_t(1) << cpos[j];
    constexpr int D = 1 << K;
    for (int r = 0; r < D; ++r) {
        uint64_t off = 0;
        for (int j = 0; j < K; ++j)
            if ((r >> (K - 1 - j)) & 1) off |= uint64_t(1) << tpos[j];
        a.tgt_off[r] = off;
    }
    for (int i = 0; i < D * D; ++i) a.u[i] = cx<R>{R(u[2 * i]), R(u[2 * i + 1])};
    constexpr int ITEMS = (K == 2 && sizeof(R) == 8) ? 1 : 2;
    const uint64_t per_block = uint64_t(kBlock) * ITEMS;
    const uint64_t blocks = (a.n_groups + per_block - 1) / per_block;
    if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
    const char *name = K == 0 ? "phase" : (K == 1 ? "gate1" : "gate2");
    const int tok = timer_begin(name, s);
    hipLaunchKernelGGL((k_small_gate<R, K, ITEMS>), dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                       a);
    timer_end(tok, s);
    return hipGetLastError();
}

template <typename R>
hipError_t small_gate_dispatch(void *amp, int n, int k, const int *tpos, int n_ctrl,
                               const int *cpos, const int *cval, const double *u,
                               hipStream_t s) {
    switch (k) {
    case 0: return small_gate_typed<R, 0>(amp, n, tpos, n_ctrl, cpos, cval, u, s);
    case 1: return small_gate_typed<R, 1>(amp, n, tpos, n_ctrl, cpos, cval, u, s);
    case 2: return small_gate_typed<R, 2>(amp, n, tpos, n_ctrl, cpos, cval, u, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t fused_valu_typed(void *amp, int n, const FusedGeom &g, const void *u_dev,
                            hipStream_t s) {
    if (g.k < 1 || g.k > 5 || g.n_sel < 0 || g.n_sel > kMaxSel) return hipErrorInvalidValue;
    const uint64_t n_cols = uint64_t(1) << (n - g.k);
    const unsigned grid = grid_for(n_cols, kBlock, kStreamGridCap);
    auto *A = static_cast<cx<R> *>(amp);
    auto *U = static_cast<const cx<R> *>(u_dev);
    const size_t lds = (size_t(1) << g.n_sel) * (size_t(1) << (2 * g.k)) * sizeof(cx<R>);
    const int tok = timer_begin(sizeof(R) == 8 ? "fused_valu_c128" : "fused_valu_c64", s);
    switch (g.k) {
    case 1: hipLaunchKernelGGL((k_fused_valu<R, 1>), dim3(grid), dim3(kBlock), lds, s, A, n_cols, g, U); break;
    case 2: hipLaunchKernelGGL((k_fused_valu<R, 2>), dim3(grid), dim3(kBlock), lds, s, A, n_cols, g, U); break;
    case 3: hipLaunchKernelGGL((k_fused_valu<R, 3>), dim3(grid), dim3(kBlock), lds, s, A, n_cols, g, U); break;
    case 4: hipLaunchKernelGGL((k_fused_valu<R, 4>), dim3(grid), dim3(kBlock), lds, s, A, n_cols, g, U); break;
    case 5: hipLaunchKernelGGL((k_fused_valu<R, 5>), dim3(grid), dim3(kBlock), lds, s, A, n_cols, g, U); break;
    default: timer_end(tok, s); return hipErrorInvalidValue;
    }
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_init(void *amp, int dtype, int n, uint64_t basis, hipStream_t s) {
    const uint64_t count = uint64_t(1) << n;
    const unsigned grid = grid_for(count, kBlock * 4, kStreamGridCap);
    const int tok = timer_begin("init", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_init_basis<float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(amp), count, basis);
    else
        hipLaunchKernelGGL((k_init_basis<double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(amp), count, basis);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, int dt_dst, const void *src, int dt_src, uint64_t count,
                       hipStream_t s) {
    const size_t elem = dt_src == QC_C64 ? 8 : 16;
    const bool aligned = ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0;
    if (dt_dst == dt_src && aligned && (count * elem) % 16 == 0) {
        const uint64_t units = count * elem / 16;
        const uint64_t chunks = (units + uint64_t(kBlock) * kCopyUnits - 1) / (uint64_t(kBlock) * kCopyUnits);
        const unsigned grid = unsigned(chunks < (uint64_t(1) << 22) ? chunks : (uint64_t(1) << 22));
        const int tok = timer_begin("copy", s);
        hipLaunchKernelGGL(k_copy_vec, dim3(grid), dim3(kBlock), 0, s,
                           static_cast<floatx4_t *>(dst), static_cast<const floatx4_t *>(src), units);
        timer_end(tok, s);
        return hipGetLastError();
    }
    const unsigned grid = grid_for(count, kBlock * 4, kStreamGridCap);
    const int tok = timer_begin("copy", s);
    if (dt_dst == QC_C64 && dt_src == QC_C64)
        hipLaunchKernelGGL((k_copy<float, float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(dst), static_cast<const cx<float> *>(src), count);
    else if (dt_dst == QC_C64 && dt_src == QC_C128)
        hipLaunchKernelGGL((k_copy<float, double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(dst), static_cast<const cx<double> *>(src), count);
    else if (dt_dst == QC_C128 && dt_src == QC_C64)
        hipLaunchKernelGGL((k_copy<double, float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(dst), static_cast<const cx<float> *>(src), count);
    else
        hipLaunchKernelGGL((k_copy<double, double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(dst), static_cast<const cx<double> *>(src), count);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_small_gate(void *amp, int dtype, int n, int k, const int *tpos, int n_ctrl,
                             const int *cpos, const int *cval, const double *u, hipStream_t s) {
    if (k + n_ctrl > n || k + n_ctrl > kMaxPos) return hipErrorInvalidValue;
    if (dtype == QC_C64) return small_gate_dispatch<float>(amp, n, k, tpos, n_ctrl, cpos, cval, u, s);
    return small_gate_dispatch<double>(amp, n, k, tpos, n_ctrl, cpos, cval, u, s);
}

hipError_t launch_phase(void *amp, int dtype, int n, int m, const int *pos, const int *val,
                        double phase_re, double phase_im, hipStream_t s) {
    const double u[2] = {phase_re, phase_im};
    return launch_small_gate(amp, dtype, n, 0, nullptr, m, pos, val, u, s);
}

hipError_t launch_fused_valu(void *amp, int dtype, int n, const FusedGeom &g, const void *u_dev,
                             hipStream_t s) {
    if (dtype == QC_C64) return fused_valu_typed<float>(amp, n, g, u_dev, s);
    return fused_valu_typed<double>(amp, n, g, u_dev, s);
}

}  // namespace qcx
