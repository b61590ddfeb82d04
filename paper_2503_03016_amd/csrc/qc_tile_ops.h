// Device-side interpreter of a run of gates on a state tile held in LDS
// (shared by the tile-run kernel, the batched persistent kernel and the
// tiled adjoint kernel).
//
// Every gate is the map psi -> (I_l (x) U' (x) I_r) psi of QCLAB section
// 3.2 restricted to the 2^m amplitudes of the tile; positions are
// compressed tile positions, controls outside the tile are tested once per
// tile against the tile's base index.
#pragma once

#include "qc_internal.h"

namespace qcx {
namespace tile {

constexpr int kBlock = 256;

template <typename R>
__device__ inline cx<R> ld_u(const double *u, int i) {
    return cx<R>{R(u[2 * i]), R(u[2 * i + 1])};
}

// Apply one op to the tile in `lds` (no barrier).  Ops whose conditions on
// bits outside the tile fail are skipped by the caller.
template <typename R>
__device__ inline void apply_one(cx<R> *lds, int m, const TileOp &op) {
    const int T = 1 << m;
    switch (op.kind) {
    case TILE_DENSE1: {
        const int b = op.b0;
        const cx<R> u0 = ld_u<R>(op.u, 0), u1 = ld_u<R>(op.u, 1), u2 = ld_u<R>(op.u, 2),
                    u3 = ld_u<R>(op.u, 3);
        for (int g = threadIdx.x; g < (T >> 1); g += kBlock) {
            const uint32_t i0 = uint32_t(insert_zero(uint64_t(g), b));
            if ((i0 & op.cmask_lo) != op.cval_lo) continue;
            const uint32_t i1 = i0 | (1u << b);
            const cx<R> a0 = lds[i0], a1 = lds[i1];
            const cx<R> z{R(0), R(0)};
            lds[i0] = cfma(u1, a1, cfma(u0, a0, z));
            lds[i1] = cfma(u3, a1, cfma(u2, a0, z));
        }
    } break;
    case TILE_DENSE2: {
        const int b0 = op.b0, b1 = op.b1;
        const int lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
        const uint32_t o1 = 1u << b1, o2 = 1u << b0;   // local index r = 2 bit(b0) + bit(b1)
        for (int g = threadIdx.x; g < (T >> 2); g += kBlock) {
            const uint32_t base = uint32_t(insert_zero(insert_zero(uint64_t(g), lo), hi));
            if ((base & op.cmask_lo) != op.cval_lo) continue;
            const uint32_t idx[4] = {base, base | o1, base | o2, base | o1 | o2};
            cx<R> a[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = lds[idx[r]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                cx<R> acc{R(0), R(0)};
#pragma unroll
                for (int c = 0; c < 4; ++c) acc = cfma(ld_u<R>(op.u, 4 * r + c), a[c], acc);
                lds[idx[r]] = acc;
            }
        }
    } break;
    case TILE_PHASE: {
        const cx<R> ph = ld_u<R>(op.u, 0);
        for (int i = threadIdx.x; i < T; i += kBlock)
            if ((uint32_t(i) & op.cmask_lo) == op.cval_lo) lds[i] = cmul(ph, lds[i]);
    } break;
    case TILE_DIAG1: {  // amp *= d[bit b]
        const cx<R> d0 = ld_u<R>(op.u, 0), d1 = ld_u<R>(op.u, 1);
        const int b = op.b0;
        for (int i = threadIdx.x; i < T; i += kBlock)
            if ((uint32_t(i) & op.cmask_lo) == op.cval_lo)
                lds[i] = cmul(((i >> b) & 1) ? d1 : d0, lds[i]);
    } break;
    default: break;   // TILE_GRAD and unknown kinds do not change the state
    }
}

// Apply a run of ops, one workgroup barrier per op.
template <typename R>
__device__ inline void apply_ops(cx<R> *lds, int m, uint64_t tile_base, const TileOp *ops,
                                 int n_ops) {
    for (int o = 0; o < n_ops; ++o) {
        const TileOp &op = ops[o];
        if ((tile_base & op.cmask_hi) != op.cval_hi) continue;   // uniform per tile
        apply_one<R>(lds, m, op);
        __syncthreads();
    }
}

// address offset of compressed tile index j
__device__ inline uint64_t deposit(uint32_t j, const uint8_t *pos, int m) {
    uint64_t off = 0;
    for (int b = 0; b < m; ++b)
        if ((j >> b) & 1) off |= uint64_t(1) << pos[b];
    return off;
}

}  // namespace tile
}  // namespace qcx
