// LDS tile kernel: one pass over the state applies a whole run of gates.
//
// A tile is the set of 2^m amplitudes that share every index bit outside a
// chosen set P of m "tile bits" (P always contains the lowest bits, so a
// tile is a union of contiguous runs in HBM).  Every gate of the run has its
// non-diagonal action (its targets) inside P; diagonal gates and controls
// may sit on any bit, because every bit of every amplitude of a tile is
// known once the tile is resident.  The kernel loads the tile into LDS with
// coalesced loads, applies the gates one after the other (one barrier per
// gate, see qc_tile_ops.h), and writes the tile back: a run of G gates costs
// one HBM read and one HBM write of the state instead of G of each.
#include "qc_rt_ops.h"
#include "qc_tile_ops.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

using tile::kBlock;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_tile_run(cx<R> *amp, const TileArgs a,
                                                     const TileOp *ops) {
    extern __shared__ unsigned char smem[];
    __shared__ TileOp op_slot[2];
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    const int T = 1 << a.m;
    // the low 8 compressed bits of this thread's elements are fixed
    const uint64_t off_lo =
        tile::deposit(uint32_t(threadIdx.x) & (T - 1), a.pos, a.m < tile::kLoBits ? a.m : tile::kLoBits);
    const uint64_t mask = tile::hi_mask(a.pos, a.m);
    for (uint64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
        const uint64_t base = insert_zeros(t, a.pos, a.m);
        tile::tile_load<R>(lds, amp, base, off_lo, mask, T);
        __syncthreads();
        tile::apply_ops<R>(lds, a.m, base, ops, a.n_ops, op_slot);
        tile::tile_store<R>(amp, lds, base, off_lo, mask, T);
        __syncthreads();
    }
}

// Register-resident tile run: each thread loads its 2^RB elements of the
// tile straight into registers (its offsets under the load layout), the op
// program runs on the registers (LDS only for RT_REMAP), and the elements
// are stored under the final layout.
template <typename R, int RB, bool PF>
__device__ __forceinline__ void rt_run_body(cx<R> *__restrict__ amp, const RtArgs &a,
                                            const RtOp *__restrict__ ops,
                                            const unsigned char *__restrict__ tabs) {
    constexpr int E = 1 << RB;
    extern __shared__ unsigned char smem[];
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    const uint32_t tid = threadIdx.x;
    const bool act = tid < (1u << a.tb);
    // the lane tables go to LDS behind the exchange area, once
    unsigned char *ltab = smem + (size_t(1) << a.m) * sizeof(cx<R>);
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
    // PF: the next tile's loads are issued before the current tile's ops run
    // (a second register set; the ops issue no vector memory instructions,
    // so nothing waits for those loads before the next tile starts)
    cx<R> nx[E];
    uint64_t t = blockIdx.x;
    if (PF && act && t < a.n_tiles) {
        const cx<R> *src = amp + insert_zeros(t, a.pos, a.m) + thr_ld;
#pragma unroll
        for (int e = 0; e < E; ++e) nx[e] = src[rt::reg_offset<RB>(e, a.ld_reg)];
    }
    for (; t < a.n_tiles; t += gridDim.x) {
        const uint64_t base = insert_zeros(t, a.pos, a.m);
        cx<R> v[E];
        if (PF) {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = nx[e];
            const uint64_t t2 = t + gridDim.x;
            if (act && t2 < a.n_tiles) {
                const cx<R> *src = amp + insert_zeros(t2, a.pos, a.m) + thr_ld;
#pragma unroll
                for (int e = 0; e < E; ++e) nx[e] = src[rt::reg_offset<RB>(e, a.ld_reg)];
            }
        } else if (act) {
            const cx<R> *src = amp + base + thr_ld;
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = src[rt::reg_offset<RB>(e, a.ld_reg)];
        }
        rt::run_ops<R, RB>(v, lds, base, tid, act, ops, a.n_ops, tb);
        if (act) {
            if (a.st_scale != 1.0) {   // uniform: the deferred Hadamard factors of the circuit
                const R sc = R(a.st_scale);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = cx<R>{v[e].re * sc, v[e].im * sc};
            }
            cx<R> *dst = amp + base + thr_st;
#pragma unroll
            for (int e = 0; e < E; ++e) dst[rt::reg_offset<RB>(e, a.st_reg)] = v[e];
        }
    }
}

// 2^12-amplitude (complex128) and 2^13-amplitude (complex64) tiles: two
// workgroups per CU, so at most 128 VGPRs
template <typename R, int RB, bool PF>
__global__ __launch_bounds__(rt::kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_rt_run(cx<R> *__restrict__ amp, const RtArgs a, const RtOp *__restrict__ ops,
              const unsigned char *__restrict__ tabs) {
    rt_run_body<R, RB, PF>(amp, a, ops, tabs);
}

// wide complex128 tiles (2^13 amplitudes, 16 per thread): the 128 KiB
// exchange area leaves one workgroup per CU, whose two wavefronts per SIMD
// may take the whole register file (the prefetch set included)
template <typename R, int RB, bool PF>
__global__ __launch_bounds__(rt::kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_rt_run_wide(cx<R> *__restrict__ amp, const RtArgs a, const RtOp *__restrict__ ops,
                   const unsigned char *__restrict__ tabs) {
    rt_run_body<R, RB, PF>(amp, a, ops, tabs);
}

}  // namespace

hipError_t launch_rt_run(void *amp, int dtype, const RtArgs &a, const RtOp *ops_dev,
                         const unsigned char *tabs_dev, hipStream_t s) {
    const int rb = rt_reg_bits(dtype, a.m);
    if (a.m < rb || a.m > rb + kRtMaxTB || a.tb != a.m - rb || a.m > kTileMaxBits)
        return hipErrorInvalidValue;
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const bool wide = dtype == QC_C128 && rb == 4;
    if ((size_t(1) << a.m) * elem > (wide ? 131072u : 65536u) || a.lds_tab_bytes % 16 ||
        a.lds_tab_bytes > 16384)
        return hipErrorInvalidValue;
    const size_t lds = (size_t(1) << a.m) * elem + a.lds_tab_bytes;
    uint64_t grid = a.n_tiles;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint64_t cap = uint64_t(cus) * uint64_t(wide ? 1 : knob(QC_KNOB_TILE_WG_PER_CU));
    if (grid > cap) grid = cap;
    const unsigned threads = 1u << (a.tb < 6 ? 6 : a.tb);
    const int tok = timer_begin(dtype == QC_C64 ? "rt_run_c64" : "rt_run_c128", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_rt_run<float, 4, true>), dim3(unsigned(grid)), dim3(threads), lds, s,
                           static_cast<cx<float> *>(amp), a, ops_dev, tabs_dev);
    else if (wide)
        hipLaunchKernelGGL((k_rt_run_wide<double, 4, true>), dim3(unsigned(grid)), dim3(threads), lds,
                           s, static_cast<cx<double> *>(amp), a, ops_dev, tabs_dev);
    else
        hipLaunchKernelGGL((k_rt_run<double, 3, false>), dim3(unsigned(grid)), dim3(threads), lds, s,
                           static_cast<cx<double> *>(amp), a, ops_dev, tabs_dev);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_tile_run(void *amp, int dtype, int n, const TileArgs &a, const TileOp *ops_dev,
                           hipStream_t s) {
    if (a.m < 1 || a.m > n || a.m > kTileMaxBits) return hipErrorInvalidValue;
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t lds = (size_t(1) << a.m) * elem;
    if (lds > 131072) return hipErrorInvalidValue;   // 2^13 complex128 amplitudes
    uint64_t grid = a.n_tiles;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const uint64_t cap = uint64_t(cus) * uint64_t(knob(QC_KNOB_TILE_WG_PER_CU));
    if (grid > cap) grid = cap;
    const int tok = timer_begin(dtype == QC_C64 ? "tile_run_c64" : "tile_run_c128", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_tile_run<float>), dim3(unsigned(grid)), dim3(kBlock), lds, s,
                           static_cast<cx<float> *>(amp), a, ops_dev);
    else
        hipLaunchKernelGGL((k_tile_run<double>), dim3(unsigned(grid)), dim3(kBlock), lds, s,
                           static_cast<cx<double> *>(amp), a, ops_dev);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
