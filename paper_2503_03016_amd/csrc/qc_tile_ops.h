// Device-side interpreter of a run of gates on a state tile held in LDS
// (shared by the tile-run kernel, the batched persistent kernel and the
// tiled adjoint kernel).
//
// Every gate is the map psi -> (I_l (x) U' (x) I_r) psi of QCLAB section
// 3.2 restricted to the 2^m amplitudes of the tile; positions are
// compressed tile positions, controls outside the tile are tested once per
// tile against the tile's base index.
//
// Each thread handles kItems independent amplitude groups per step, all
// loads first, so the LDS latency of one group is hidden behind the others.
#pragma once

#include "qc_internal.h"

namespace qcx {
namespace tile {

constexpr int kBlock = 512;     // threads per workgroup of the tile kernels
constexpr int kLoBits = 9;      // log2(kBlock)
constexpr int kLoadBatch = 8;   // tile elements a thread loads before waiting for them
constexpr int kItems = 4;       // independent groups per thread per step

template <typename R>
__device__ inline cx<R> ld_u(const double *u, int i) {
    return cx<R>{R(u[2 * i]), R(u[2 * i + 1])};
}

__device__ inline uint32_t ins0(uint32_t g, int p) {
    return ((g >> p) << (p + 1)) | (g & ((1u << p) - 1u));
}

// Values every lane holds the same (op fields read from LDS), moved to
// scalar registers so that they take no vector registers.
__device__ inline uint32_t uniform(uint32_t x) { return uint32_t(__builtin_amdgcn_readfirstlane(int(x))); }
__device__ inline float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ inline double uniform(double x) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// TILE_KRON with G matrices: one group of 2^G amplitudes per thread per
// step, loaded once; matrix j acts on the pairs that differ in bit j of the
// local index.  Bit positions and matrix entries are kept in scalar
// registers.
template <typename R, int G>
__device__ inline void apply_kron(cx<R> *lds, int m, const TileOp &op) {
    constexpr int D = 1 << G;
    const uint32_t bits = uniform(uint32_t(op.b1));
    int bit[G];
#pragma unroll
    for (int j = 0; j < G; ++j) bit[j] = (bits >> (5 * j)) & 31;
    uint32_t off[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        off[r] = 0;
#pragma unroll
        for (int j = 0; j < G; ++j)
            if ((r >> j) & 1) off[r] |= 1u << bit[j];
    }
    cx<R> um[G][4];
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            um[j][e] = cx<R>{uniform(R(op.u[8 * j + 2 * e])), uniform(R(op.u[8 * j + 2 * e + 1]))};
    const cx<R> z{R(0), R(0)};
    const int ngroups = (1 << m) >> G;
    for (int grp = threadIdx.x; grp < ngroups; grp += kBlock) {
        uint32_t base = uint32_t(grp);
#pragma unroll
        for (int j = 0; j < G; ++j) base = ins0(base, bit[j]);   // ascending positions
        cx<R> a[D];
#pragma unroll
        for (int r = 0; r < D; ++r) a[r] = lds[base | off[r]];
#pragma unroll
        for (int j = 0; j < G; ++j)
#pragma unroll
            for (int r = 0; r < D; ++r)
                if (!((r >> j) & 1)) {
                    const cx<R> a0 = a[r], a1 = a[r | (1 << j)];
                    a[r] = cfma(um[j][1], a1, cfma(um[j][0], a0, z));
                    a[r | (1 << j)] = cfma(um[j][3], a1, cfma(um[j][2], a0, z));
                }
#pragma unroll
        for (int r = 0; r < D; ++r) lds[base | off[r]] = a[r];
    }
}

// Apply one op to the tile in `lds` (no barrier).  Ops whose conditions on
// bits outside the tile fail are skipped by the caller.  KRON = false
// compiles TILE_KRON out (for kernels whose op lists are built without it,
// where its registers would lower occupancy).
template <typename R, bool KRON = true>
__device__ inline void apply_one(cx<R> *lds, int m, const TileOp &op) {
    const int T = 1 << m;
    const uint32_t cm = op.cmask_lo, cv = op.cval_lo;
    switch (op.kind) {
    case TILE_DENSE1: {
        const int b = op.b0;
        const uint32_t bit = 1u << b;
        const cx<R> u0 = ld_u<R>(op.u, 0), u1 = ld_u<R>(op.u, 1), u2 = ld_u<R>(op.u, 2),
                    u3 = ld_u<R>(op.u, 3);
        const int npairs = T >> 1;
        for (int g0 = threadIdx.x; g0 < npairs; g0 += kBlock * kItems) {
            uint32_t i0[kItems];
            bool ok[kItems];
            cx<R> a0[kItems], a1[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const int g = g0 + k * kBlock;
                i0[k] = ins0(uint32_t(g), b);
                ok[k] = g < npairs && (i0[k] & cm) == cv;
                if (ok[k]) {
                    a0[k] = lds[i0[k]];
                    a1[k] = lds[i0[k] | bit];
                }
            }
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                if (!ok[k]) continue;
                const cx<R> z{R(0), R(0)};
                lds[i0[k]] = cfma(u1, a1[k], cfma(u0, a0[k], z));
                lds[i0[k] | bit] = cfma(u3, a1[k], cfma(u2, a0[k], z));
            }
        }
    } break;
    case TILE_DENSE2: {
        const int b0 = op.b0, b1 = op.b1;
        const int lo = b0 < b1 ? b0 : b1, hi = b0 < b1 ? b1 : b0;
        const uint32_t o1 = 1u << b1, o2 = 1u << b0;   // local index r = 2 bit(b0) + bit(b1)
        const int ngroups = T >> 2;
        for (int g0 = threadIdx.x; g0 < ngroups; g0 += kBlock * 2) {
            uint32_t base[2];
            bool ok[2];
            cx<R> a[2][4];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int g = g0 + k * kBlock;
                base[k] = ins0(ins0(uint32_t(g), lo), hi);
                ok[k] = g < ngroups && (base[k] & cm) == cv;
                if (ok[k]) {
                    a[k][0] = lds[base[k]];
                    a[k][1] = lds[base[k] | o1];
                    a[k][2] = lds[base[k] | o2];
                    a[k][3] = lds[base[k] | o1 | o2];
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (!ok[k]) continue;
                const uint32_t idx[4] = {base[k], base[k] | o1, base[k] | o2, base[k] | o1 | o2};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cx<R> acc{R(0), R(0)};
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc = cfma(ld_u<R>(op.u, 4 * r + c), a[k][c], acc);
                    lds[idx[r]] = acc;
                }
            }
        }
    } break;
    case TILE_PHASE: {
        const cx<R> ph = ld_u<R>(op.u, 0);
        for (int i0 = threadIdx.x; i0 < T; i0 += kBlock * kItems) {
            cx<R> v[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const int i = i0 + k * kBlock;
                if (i < T && (uint32_t(i) & cm) == cv) v[k] = lds[i];
            }
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const int i = i0 + k * kBlock;
                if (i < T && (uint32_t(i) & cm) == cv) lds[i] = cmul(ph, v[k]);
            }
        }
    } break;
    case TILE_DIAG1: {  // amp *= d[bit b]
        const cx<R> d0 = ld_u<R>(op.u, 0), d1 = ld_u<R>(op.u, 1);
        const int b = op.b0;
        for (int i0 = threadIdx.x; i0 < T; i0 += kBlock * kItems) {
            cx<R> v[kItems];
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const int i = i0 + k * kBlock;
                if (i < T && (uint32_t(i) & cm) == cv) v[k] = lds[i];
            }
#pragma unroll
            for (int k = 0; k < kItems; ++k) {
                const int i = i0 + k * kBlock;
                if (i < T && (uint32_t(i) & cm) == cv) lds[i] = cmul(((i >> b) & 1) ? d1 : d0, v[k]);
            }
        }
    } break;
    case TILE_KRON:
        if constexpr (KRON) {
            if (op.b0 == 2) apply_kron<R, 2>(lds, m, op);
            else if (op.b0 == 3) apply_kron<R, 3>(lds, m, op);
        }
        break;
    default: break;   // TILE_GRAD, TILE_PHASES, TILE_DENSE1_PHASES, the fan ops (see apply_ops), unknown kinds
    }
}

// TILE_PHASES: product of the diagonal terms whose conditions hold.  All
// in-tile conditions of an op lie in the bit set U = op.b1 (at most
// kPhaseTableBits bits, enforced when the op is built), so the phase of an
// amplitude depends only on its bits in U: a table of 2^|U| products is
// built once per op (one entry per thread) and every amplitude then takes
// one table lookup and one complex product.
// compact the bits of i that lie in mask u (ascending) into the low bits
__device__ inline uint32_t extract_bits(uint32_t i, uint32_t u) {
    uint32_t e = 0, k = 0;
    while (u) {
        const uint32_t b = uint32_t(__builtin_ctz(u));
        e |= ((i >> b) & 1u) << k;
        ++k;
        u &= u - 1;
    }
    return e;
}
// inverse of extract_bits: spread the low bits of e over the positions of u
__device__ inline uint32_t deposit_bits(uint32_t e, uint32_t u) {
    uint32_t i = 0, k = 0;
    while (u) {
        const uint32_t b = uint32_t(__builtin_ctz(u));
        i |= ((e >> k) & 1u) << b;
        ++k;
        u &= u - 1;
    }
    return i;
}

// Element i = threadIdx.x + kBlock g of a tile has table index
// e_lo | hix[g]: e_lo from the thread's low kLoBits bits (fixed per thread),
// hix[g] from the group number g (the same for every lane), so that no lane
// compacts bits per element.
constexpr int kPhaseGroups = 1 << (kTileMaxBits - kLoBits);
static_assert((1 << kPhaseTableBits) <= kBlock / 2 && (1 << kPhaseTableBits) % 64 == 0,
              "table entries and group indices use disjoint wavefronts");
static_assert(kPhaseGroups <= kBlock / 2, "one group index per thread");

// Fill `tab` (2^|U| entries, LDS) and `hix` (one entry per element group)
// for the first n_terms terms of op, which test the tile bits U; returns
// false when no term is live for this tile (the op is the identity there).
// Caller syncs before using the tables.
template <typename R>
__device__ inline R lane_value(R x, int lane);
template <>
__device__ inline float lane_value(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
template <>
__device__ inline double lane_value(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

template <typename R>
__device__ inline bool phases_table(cx<R> *tab, uint32_t *hix, int m, uint64_t tile_base,
                                    const TileOp &op, int n_terms, uint32_t U_in) {
    static_assert(kTilePhaseTerms <= 64, "one term per lane");
    const int nt = int(uniform(uint32_t(n_terms)));
    const uint32_t U = uniform(U_in);
    // lane t of every wavefront loads term t (all terms at once, no chain
    // of dependent LDS reads); the term's fields then reach the other lanes
    // through readlane
    const int lane = int(threadIdx.x & 63);
    const int tl = lane < kTilePhaseTerms ? lane : 0;
    const uint32_t ml = op.pm_lo[tl], vl = op.pv_lo[tl];
    const R pr = R(op.u[2 * tl]), pi = R(op.u[2 * tl + 1]);
    const bool ok = lane < nt && (tile_base & op.pm_hi[tl]) == op.pv_hi[tl];
    // terms whose out-of-tile conditions hold for this tile
    const uint32_t live = uniform(uint32_t(__ballot(ok)));
    if (!live) return false;
    const uint32_t entries = 1u << __builtin_popcount(U);
    const uint32_t e = threadIdx.x;
    // whole wavefronts enter (the condition is the same for its 64 lanes):
    // readlane takes the term from a lane that must have computed it, so no
    // lane may be switched off here; lanes past the table build a dummy entry
    if ((e & ~63u) < entries) {
        const uint32_t i = deposit_bits(e < entries ? e : 0u, U);
        cx<R> f{R(1), R(0)};
#pragma unroll
        for (int t = 0; t < kTilePhaseTerms; ++t) {
            if (!((live >> t) & 1u)) continue;   // uniform
            const uint32_t mt = uint32_t(__builtin_amdgcn_readlane(int(ml), t));
            const uint32_t vt = uint32_t(__builtin_amdgcn_readlane(int(vl), t));
            const cx<R> p{lane_value(pr, t), lane_value(pi, t)};
            if ((i & mt) == vt) f = cmul(f, p);
        }
        if (e < entries) tab[e] = f;
    } else if (e >= uint32_t(kBlock / 2)) {
        const uint32_t g = e - uint32_t(kBlock / 2);
        const uint32_t groups = m > kLoBits ? 1u << (m - kLoBits) : 1u;
        if (g < groups) hix[g] = extract_bits(g, U >> kLoBits) << __builtin_popcount(U & (kBlock - 1));
    }
    return true;
}

// Multiply every amplitude of the tile by its table entry.
template <typename R>
__device__ inline void phases_apply(cx<R> *lds, int m, const cx<R> *tab, const uint32_t *hix,
                                    uint32_t U) {
    const int T = 1 << m;
    const uint32_t e_lo = extract_bits(threadIdx.x & (kBlock - 1), U & (kBlock - 1));
    for (int i0 = threadIdx.x, g0 = 0; i0 < T; i0 += kBlock * kItems, g0 += kItems) {
        cx<R> v[kItems], f[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int i = i0 + k * kBlock;
            if (i < T) {   // then g0 + k < max(T / kBlock, 1)
                v[k] = lds[i];
                f[k] = tab[e_lo | hix[g0 + k]];
            }
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int i = i0 + k * kBlock;
            if (i < T) lds[i] = cmul(f[k], v[k]);
        }
    }
}

// LDS of a TILE_PHASES op: the product table and the group indices
template <typename R>
struct PhaseTables {
    cx<R> tab[1 << kPhaseTableBits];
    uint32_t hix[kPhaseGroups];
};

template <typename R>
__device__ inline void apply_phases(cx<R> *lds, int m, uint64_t tile_base, const TileOp &op,
                                    PhaseTables<R> &pt) {
    const bool any = phases_table<R>(pt.tab, pt.hix, m, tile_base, op, op.b0, uint32_t(op.b1));
    __syncthreads();
    if (any) phases_apply<R>(lds, m, pt.tab, pt.hix, uint32_t(op.b1));
}

// TILE_DENSE1_PHASES: pair (i0, i1 = i0 | 2^b) gets the matrix, then each
// element its table entry.  Thread t takes the pairs g = t + kBlock k; the
// low kLoBits bits of i0 = ins0(g, b) and of i1 depend on t only, so their
// part of the table index is found once per thread, and the rest is the
// group entry hix[i >> kLoBits].
template <typename R>
__device__ inline void apply_dense1_phases(cx<R> *lds, int m, uint64_t tile_base, const TileOp &op,
                                           PhaseTables<R> &pt) {
    const uint32_t U = uint32_t(op.b1);
    const bool any = phases_table<R>(pt.tab, pt.hix, m, tile_base, op, op.pad, U);   // uniform
    __syncthreads();
    const int T = 1 << m;
    const int b = op.b0;
    const uint32_t bit = 1u << b;
    const cx<R> u0 = ld_u<R>(op.u1, 0), u1 = ld_u<R>(op.u1, 1), u2 = ld_u<R>(op.u1, 2),
                u3 = ld_u<R>(op.u1, 3);
    const uint32_t lo = ins0(threadIdx.x, b) & (kBlock - 1);
    const uint32_t e0_lo = extract_bits(lo, U & (kBlock - 1));
    const uint32_t e1_lo = extract_bits((lo | bit) & (kBlock - 1), U & (kBlock - 1));
    const int npairs = T >> 1;
    for (int g0 = threadIdx.x; g0 < npairs; g0 += kBlock * kItems) {
        // complex64: every LDS read of the step (amplitudes and table
        // entries) is issued before any is used; complex128 reads the table
        // entries where they are used (holding them too would take the
        // batch kernel past 128 registers)
        constexpr bool kEarly = sizeof(R) == sizeof(float);
        uint32_t i0[kItems];
        cx<R> a0[kItems], a1[kItems], f0[kItems], f1[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int g = g0 + k * kBlock;
            i0[k] = ins0(uint32_t(g), b);
            if (g < npairs) {
                a0[k] = lds[i0[k]];
                a1[k] = lds[i0[k] | bit];
                if (kEarly && any) {
                    f0[k] = pt.tab[e0_lo | pt.hix[i0[k] >> kLoBits]];
                    f1[k] = pt.tab[e1_lo | pt.hix[(i0[k] | bit) >> kLoBits]];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (g0 + k * kBlock >= npairs) continue;
            const cx<R> z{R(0), R(0)};
            cx<R> v0 = cfma(u1, a1[k], cfma(u0, a0[k], z));
            cx<R> v1 = cfma(u3, a1[k], cfma(u2, a0[k], z));
            if (any) {
                if (!kEarly) {
                    f0[k] = pt.tab[e0_lo | pt.hix[i0[k] >> kLoBits]];
                    f1[k] = pt.tab[e1_lo | pt.hix[(i0[k] | bit) >> kLoBits]];
                }
                v0 = cmul(f0[k], v0);
                v1 = cmul(f1[k], v1);
            }
            lds[i0[k]] = v0;
            lds[i0[k] | bit] = v1;
        }
    }
}

// TILE_FAN / TILE_DENSE1_FAN.  The phase of an amplitude with the target
// bit set factorizes: K (terms on the target alone, and the out-of-tile
// controls the tile has set) times the phases of its set control bits
// below kLoBits (fixed per thread: the pairs a thread takes share their low
// bits; from two small tables, over bits 0..5 and 6..8) times those of its
// set control bits above (fixed per group of kBlock elements: one entry per
// group, K included).  The tables are built by the first two wavefronts.
// No table over all the control bits and no limit on their number.
constexpr int kFanGroups = 1 << (13 - kLoBits);   // tiles hold at most 2^13 amplitudes

// LDS of a fan op: the group factors (K included) and two tables of the
// low-bit factor: lo6[e] over control bits 0..5, lo3[e] over bits 6..8
template <typename R>
struct FanTables {
    cx<R> h[kFanGroups];
    cx<R> lo6[64], lo3[8];
};

template <typename R, bool DENSE>
__device__ inline void apply_fan(cx<R> *lds, int m, uint64_t tile_base, const TileOp &op,
                                 FanTables<R> &ft) {
    static_assert(kLoBits == 9, "the low-bit factor tables cover 6 + 3 bits");
    const int T = 1 << m;
    const int t = op.b0;
    const uint32_t bit = 1u << t;
    const uint32_t cm = uniform(uint32_t(op.b1));
    if (threadIdx.x < 64) {   // wavefront 0: K, the group factors, lo6
        // K: lane k takes out-of-tile control k, then a butterfly over 16
        // lanes multiplies them; lane 0's product is used
        const int nh = int(uniform(uint32_t(op.pad)));
        const int lane = int(threadIdx.x);
        const int kl = lane < kTilePhaseTerms ? lane : 0;
        const uint64_t fm = op.fan_mask[kl];
        cx<R> f{R(1), R(0)};
        if (lane < nh && (tile_base & fm) == fm) f = cx<R>{R(op.fan_ph[2 * kl]), R(op.fan_ph[2 * kl + 1])};
        static_assert(kTilePhaseTerms == 16, "one butterfly over 16 lanes");
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const cx<R> o{__shfl_xor(f.re, off, 64), __shfl_xor(f.im, off, 64)};
            f = cmul(f, o);
        }
        cx<R> K{lane_value(f.re, 0), lane_value(f.im, 0)};
        K = cmul(K, ld_u<R>(op.u, t));
        const int groups = m > kLoBits ? 1 << (m - kLoBits) : 1;
        if (lane < groups) {
            cx<R> h = K;
            for (int c = kLoBits; c < m; ++c)
                if (((cm >> c) & 1u) && ((lane >> (c - kLoBits)) & 1)) h = cmul(h, ld_u<R>(op.u, c));
            ft.h[lane] = h;
        }
        cx<R> p{R(1), R(0)};
#pragma unroll
        for (int c = 0; c < 6; ++c)
            if (((cm >> c) & 1u) && ((lane >> c) & 1)) p = cmul(p, ld_u<R>(op.u, c));
        ft.lo6[lane] = p;
    } else if (threadIdx.x < 72) {   // lo3
        const int e = int(threadIdx.x) - 64;
        cx<R> p{R(1), R(0)};
#pragma unroll
        for (int c = 6; c < kLoBits; ++c)
            if (((cm >> c) & 1u) && ((e >> (c - 6)) & 1)) p = cmul(p, ld_u<R>(op.u, c));
        ft.lo3[e] = p;
    }
    // the thread's elements with the target set share their low kLoBits bits
    const uint32_t lo1 = (ins0(threadIdx.x, t) | bit) & (kBlock - 1);
    cx<R> u0, u1, u2, u3;
    if (DENSE) {
        u0 = ld_u<R>(op.u1, 0);
        u1 = ld_u<R>(op.u1, 1);
        u2 = ld_u<R>(op.u1, 2);
        u3 = ld_u<R>(op.u1, 3);
    }
    __syncthreads();   // the fan tables
    const cx<R> flo = cmul(ft.lo6[lo1 & 63], ft.lo3[lo1 >> 6]);
    const int npairs = T >> 1;
    for (int g0 = threadIdx.x; g0 < npairs; g0 += kBlock * kItems) {
        uint32_t i1[kItems];
        cx<R> a0[kItems], a1[kItems], h[kItems];
        // every LDS read of the step (amplitudes and group factors) is
        // issued before any is used
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const int g = g0 + k * kBlock;
            i1[k] = ins0(uint32_t(g), t) | bit;
            if (g < npairs) {
                if (DENSE) a0[k] = lds[i1[k] ^ bit];
                a1[k] = lds[i1[k]];
                h[k] = ft.h[i1[k] >> kLoBits];
            }
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (g0 + k * kBlock >= npairs) continue;
            const cx<R> ph = cmul(flo, h[k]);
            if (DENSE) {
                const cx<R> z{R(0), R(0)};
                lds[i1[k] ^ bit] = cfma(u1, a1[k], cfma(u0, a0[k], z));
                lds[i1[k]] = cmul(ph, cfma(u3, a1[k], cfma(u2, a0[k], z)));
            } else {
                lds[i1[k]] = cmul(ph, a1[k]);
            }
        }
    }
}

// TILE_XPERM: each thread takes its elements i (threadIdx.x + kBlock k),
// finds its partner j = i ^ f(i) and swaps the two when j > i, so every
// pair is moved by exactly one thread and no barrier is needed inside the
// op.  The gates' fields are moved to scalar registers; lane k of every
// wavefront checks the out-of-tile controls of gate k.
template <typename R>
__device__ inline void apply_xperm(cx<R> *lds, int m, uint64_t tile_base, const TileOp &op) {
    const int T = 1 << m;
    const int nt = int(uniform(uint32_t(op.b0)));
    const int lane = int(threadIdx.x & 63);
    const int kl = lane < kXpermTerms ? lane : 0;
    const bool ok = lane < nt && (tile_base & op.x_hm[kl]) == op.x_hv[kl];
    const uint32_t live = uniform(uint32_t(__ballot(ok)));
    uint32_t cm[kXpermTerms], cv[kXpermTerms], fb[kXpermTerms];
#pragma unroll
    for (int t = 0; t < kXpermTerms; ++t) {
        cm[t] = uniform(op.x_cm[t]);
        cv[t] = uniform(op.x_cv[t]);
        fb[t] = ((live >> t) & 1u) ? 1u << uniform(op.x_t[t]) : 0u;
    }
    for (int i0 = threadIdx.x; i0 < T; i0 += kBlock * kItems) {
        uint32_t j[kItems];
        cx<R> a[kItems], b[kItems];
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t i = uint32_t(i0 + k * kBlock);
            uint32_t f = 0;
#pragma unroll
            for (int t = 0; t < kXpermTerms; ++t)
                if ((i & cm[t]) == cv[t]) f |= fb[t];
            j[k] = i ^ f;
            const bool mine = i < uint32_t(T) && j[k] > i;
            a[k] = mine ? lds[i] : cx<R>{R(0), R(0)};
            b[k] = mine ? lds[j[k]] : cx<R>{R(0), R(0)};
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t i = uint32_t(i0 + k * kBlock);
            if (i < uint32_t(T) && j[k] > i) {
                lds[i] = b[k];
                lds[j[k]] = a[k];
            }
        }
    }
}

// Op staging: the op being applied is read from one of two LDS slots.
// While op o runs, the first kOpWords lanes hold op o + 1 in registers
// (a global load issued before op o starts) and write it to the other slot
// right before op o's closing barrier, so the fetch latency of the op list
// is hidden behind the work and every thread reads op fields (matrix
// entries, phase terms) from LDS.
constexpr int kOpWords = int(sizeof(TileOp) / sizeof(uint64_t));
static_assert(sizeof(TileOp) % sizeof(uint64_t) == 0, "TileOp is copied in 8-byte words");
static_assert(kOpWords <= kBlock, "one word per thread");

struct OpStage {
    uint64_t word = 0;
};

// Copy op `src` into `dst` (LDS) now; the caller places the barrier.
__device__ inline void stage_now(TileOp *dst, const TileOp *src) {
    if (threadIdx.x < kOpWords)
        reinterpret_cast<uint64_t *>(dst)[threadIdx.x] =
            reinterpret_cast<const uint64_t *>(src)[threadIdx.x];
}
// Start fetching op `src` (no wait).
__device__ inline void stage_fetch(OpStage &st, const TileOp *src) {
    if (threadIdx.x < kOpWords) st.word = reinterpret_cast<const uint64_t *>(src)[threadIdx.x];
}
// Store a fetched op into `dst` (LDS); the caller places the barrier.
__device__ inline void stage_store(const OpStage &st, TileOp *dst) {
    if (threadIdx.x < kOpWords) reinterpret_cast<uint64_t *>(dst)[threadIdx.x] = st.word;
}

// Apply a run of ops, one workgroup barrier per op.  `slot` is 2 TileOps of
// LDS owned by the caller's workgroup.
template <typename R>
__device__ inline void apply_ops(cx<R> *lds, int m, uint64_t tile_base, const TileOp *ops,
                                 int n_ops, TileOp *slot) {
    if (n_ops <= 0) return;
    __shared__ PhaseTables<R> pt;
    __shared__ FanTables<R> ft;
    stage_now(&slot[0], &ops[0]);
    __syncthreads();
    for (int o = 0; o < n_ops; ++o) {
        const TileOp &op = slot[o & 1];
        const bool next = o + 1 < n_ops;
        OpStage st;
        if (next) stage_fetch(st, &ops[o + 1]);
        if ((tile_base & op.cmask_hi) == op.cval_hi) {   // uniform per tile
            if (op.kind == TILE_PHASES) apply_phases<R>(lds, m, tile_base, op, pt);
            else if (op.kind == TILE_DENSE1_PHASES) apply_dense1_phases<R>(lds, m, tile_base, op, pt);
            else if (op.kind == TILE_FAN) apply_fan<R, false>(lds, m, tile_base, op, ft);
            else if (op.kind == TILE_DENSE1_FAN) apply_fan<R, true>(lds, m, tile_base, op, ft);
            else if (op.kind == TILE_XPERM) apply_xperm<R>(lds, m, tile_base, op);
            else apply_one<R>(lds, m, op);
        }
        if (next) stage_store(st, &slot[(o + 1) & 1]);
        __syncthreads();
    }
}

// address offset of compressed tile index j
__device__ inline uint64_t deposit(uint32_t j, const uint32_t *pos, int m) {
    uint64_t off = 0;
    for (int b = 0; b < m; ++b)
        if ((j >> b) & 1) off |= uint64_t(1) << pos[b];
    return off;
}

// Offsets of the elements j = threadIdx.x + kBlock k of a tile: the low
// kLoBits compressed bits are the thread's (deposit once), the bits above
// come from k.  D(k), the deposit of k at the tile positions kLoBits .. m-1,
// runs through the submasks of hi_mask(pos, m) in ascending order, so
// D(k + 1) = next_submask(D(k), mask): no table lookups per element.
__device__ inline uint64_t hi_mask(const uint32_t *pos, int m) {
    uint64_t mask = 0;
    for (int b = kLoBits; b < m; ++b) mask |= uint64_t(1) << pos[b];
    return mask;
}
__device__ inline uint64_t next_submask(uint64_t d, uint64_t mask) { return (d - mask) & mask; }

// Move the tile at `base` between HBM and LDS (T = 2^m elements): kLoadBatch
// loads in flight per thread before the first of them is waited for.  Every
// address formed here lies in the tile (off_lo takes the thread index modulo
// T, and the submasks stay inside the mask), so the loads are guarded only
// by the uniform k < K; the LDS writes also need j < T.
template <typename R>
__device__ inline void tile_load(cx<R> *lds, const cx<R> *amp, uint64_t base, uint64_t off_lo,
                                 uint64_t mask, int T) {
    const int K = T > kBlock ? T >> kLoBits : 1;
    uint64_t d = 0;
    for (int k0 = 0; k0 < K; k0 += kLoadBatch) {
        cx<R> v[kLoadBatch];
        uint64_t dk = d;
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            v[u] = k0 + u < K ? amp[base + off_lo + dk] : cx<R>{R(0), R(0)};
            dk = next_submask(dk, mask);
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int j = int(threadIdx.x) + (k0 + u) * kBlock;
            if (k0 + u < K && j < T) lds[j] = v[u];
        }
        d = dk;
    }
}
template <typename R>
__device__ inline void tile_store(cx<R> *amp, const cx<R> *lds, uint64_t base, uint64_t off_lo,
                                  uint64_t mask, int T) {
    const int K = T > kBlock ? T >> kLoBits : 1;
    uint64_t d = 0;
    for (int k = 0; k < K; ++k) {
        const int j = int(threadIdx.x) + k * kBlock;
        if (j < T) amp[base + off_lo + d] = lds[j];
        d = next_submask(d, mask);
    }
}

}  // namespace tile
}  // namespace qcx
