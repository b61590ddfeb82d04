// Device interpreter of register-resident tile programs (see RtOp in
// qc_internal.h).
//
// Every gate is the map psi -> (I_l (x) U' (x) I_r) psi of QCLAB section
// 3.2 restricted to one tile of 2^m amplitudes.  Each thread keeps E = 2^RB
// amplitudes of the tile in registers: v[e] is tile element
// dep_reg(e) | dep_thr(t) under the current layout.  A gate on a register
// slot pairs elements of one thread (compile-time register indices, no
// communication); diagonal ops need only the index bits of each element;
// RT_REMAP exchanges bits between register and thread slots through LDS.
// Op fields are read with uniform addresses (scalar loads).
#pragma once

#include "qc_internal.h"
#include "qc_lanes.h"

namespace qcx {
namespace rt {

constexpr int kBlock = 512;   // threads per workgroup (tiles of up to 2^(RB + 9))

// global offset of element e: its bits deposited at the positions pos[i]
template <int RB>
__device__ __forceinline__ uint64_t reg_offset(int e, const uint32_t *pos) {
    uint64_t off = 0;
#pragma unroll
    for (int i = 0; i < RB; ++i)
        if ((e >> i) & 1) off |= uint64_t(1) << pos[i];
    return off;
}

// complex entry i of an op's value array (stored in the state's precision)
template <typename R>
__device__ __forceinline__ cx<R> ldu(const double *u, int i) {
    const R *p = rt_vals<R>(u);
    return cx<R>{p[2 * i], p[2 * i + 1]};
}

template <typename R>
__device__ __forceinline__ cx<R> csel(bool c, cx<R> a, cx<R> b) {
    return cx<R>{c ? a.re : b.re, c ? a.im : b.im};
}

// elements per 128-byte row of LDS banks: log2
template <typename R>
constexpr int swz_bits() { return sizeof(R) == sizeof(float) ? 4 : 3; }

// x0' = u0 x0 + u1 x1, x1' = u2 x0 + u3 x1 on the pairs of register slot S;
// COND: only where the element condition holds (uniform per pair) and the
// thread condition tc holds.
template <typename R, int RB, int S, bool REAL, bool COND>
__device__ __forceinline__ void u1_slot(cx<R> *v, const RtOp &op, bool tc) {
    constexpr int E = 1 << RB;
    const cx<R> u0 = ldu<R>(op.u, 0), u1 = ldu<R>(op.u, 1), u2 = ldu<R>(op.u, 2),
                u3 = ldu<R>(op.u, 3);
    const uint32_t rm = op.rm, rv = op.rv;
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
        if (e0 & (1 << S)) continue;
        const int e1 = e0 | (1 << S);
        // element and thread conditions as one select (no branch per pair)
        const bool c = tc && (uint32_t(e0) & rm) == rv;
        const cx<R> a = v[e0], b = v[e1];
        cx<R> x, y;
        if (REAL) {
            x = cx<R>{u0.re * a.re + u1.re * b.re, u0.re * a.im + u1.re * b.im};
            y = cx<R>{u2.re * a.re + u3.re * b.re, u2.re * a.im + u3.re * b.im};
        } else {
            const cx<R> z{R(0), R(0)};
            x = cfma(u1, b, cfma(u0, a, z));
            y = cfma(u3, b, cfma(u2, a, z));
        }
        v[e0] = COND ? csel(c, x, a) : x;
        v[e1] = COND ? csel(c, y, b) : y;
    }
}


template <typename R, int RB, int S>
__device__ __forceinline__ void h_slot(cx<R> *v) {
    constexpr int E = 1 << RB;
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
        if (e0 & (1 << S)) continue;
        const int e1 = e0 | (1 << S);
        const cx<R> a = v[e0], b = v[e1];
        v[e0] = cx<R>{a.re + b.re, a.im + b.im};
        v[e1] = cx<R>{a.re - b.re, a.im - b.im};
    }
}


// 4x4 on register slots A (most significant bit of the local index) and B
template <typename R, int RB, int A, int B, bool COND>
__device__ __forceinline__ void u2_slots(cx<R> *v, const RtOp &op, bool tc) {
    constexpr int E = 1 << RB;
    const uint32_t rm = op.rm, rv = op.rv;
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
        if (e0 & ((1 << A) | (1 << B))) continue;
        const bool c = tc && (uint32_t(e0) & rm) == rv;
        const int idx[4] = {e0, e0 | (1 << B), e0 | (1 << A), e0 | (1 << A) | (1 << B)};
        cx<R> x[4], y[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r] = v[idx[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cx<R> acc{R(0), R(0)};
#pragma unroll
            for (int c = 0; c < 4; ++c) acc = cfma(ldu<R>(op.u, 4 * r + c), x[c], acc);
            y[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) v[idx[r]] = COND ? csel(c, y[r], x[r]) : y[r];
    }
}

template <typename R, int RB, int A, bool COND>
__device__ __forceinline__ void u2_b(cx<R> *v, const RtOp &op, bool tc) {
    switch (op.b) {
    case 0: if constexpr (A != 0) u2_slots<R, RB, A, 0, COND>(v, op, tc); break;
    case 1: if constexpr (A != 1 && RB > 1) u2_slots<R, RB, A, 1, COND>(v, op, tc); break;
    case 2: if constexpr (A != 2 && RB > 2) u2_slots<R, RB, A, 2, COND>(v, op, tc); break;
    case 3: if constexpr (A != 3 && RB > 3) u2_slots<R, RB, A, 3, COND>(v, op, tc); break;
    default: break;
    }
}

template <typename R, int RB, bool COND>
__device__ __forceinline__ void u2(cx<R> *v, const RtOp &op, bool tc) {
    switch (op.a) {
    case 0: u2_b<R, RB, 0, COND>(v, op, tc); break;
    case 1: if constexpr (RB > 1) u2_b<R, RB, 1, COND>(v, op, tc); break;
    case 2: if constexpr (RB > 2) u2_b<R, RB, 2, COND>(v, op, tc); break;
    case 3: if constexpr (RB > 3) u2_b<R, RB, 3, COND>(v, op, tc); break;
    default: break;
    }
}

// diag(d0, d1) on register slot S: the element's bit picks the factor
template <typename R, int RB, int S>
__device__ __forceinline__ void diag1_slot(cx<R> *v, cx<R> d0, cx<R> d1, bool skip0) {
    constexpr int E = 1 << RB;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if ((e >> S) & 1) v[e] = cmul(d1, v[e]);
        else if (!skip0) v[e] = cmul(d0, v[e]);   // uniform
    }
}

// diag(d0, d1) on the thread slot a: the thread's bit picks the factor
template <typename R, int RB>
__device__ __forceinline__ void diag1_thread(cx<R> *v, const RtOp &op, uint32_t tid) {
    constexpr int E = 1 << RB;
    const bool hi = (tid >> op.a) & 1u;
    const cx<R> d = csel(hi, ldu<R>(op.u, 1), ldu<R>(op.u, 0));
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(d, v[e]);
}

// Per-op lookup tables: lane tables in LDS (ltab), wave and window tables
// in memory (gtab), both at byte offsets of the program's table blob.
struct Tabs {
    const unsigned char *ltab;        // LDS copy of the lane tables
    const unsigned char *__restrict__ gtab;   // the blob in memory
    uint32_t lane, wave;              // lane number, wavefront number (uniform)
};

// bit set L of the terms whose thread and tile conditions hold
__device__ __forceinline__ uint32_t terms_live(const RtOp &op, const Tabs &tb, uint64_t base) {
    uint32_t L = reinterpret_cast<const uint32_t *>(tb.ltab + op.w[0])[tb.lane] & op.w[8 + tb.wave];
    const int nw = op.b;
#pragma unroll
    for (int j = 0; j < kRtWindows; ++j)
        if (j < nw)   // uniform
            L &= op.wt[8 * j + ((base >> op.hw[j]) & 7)];
    return L;
}

template <typename R>
__device__ __forceinline__ cx<R> negate_if(cx<R> x, uint32_t odd);
template <>
__device__ __forceinline__ cx<float> negate_if(cx<float> x, uint32_t odd) {
    const uint32_t m = odd << 31;
    return cx<float>{__uint_as_float(__float_as_uint(x.re) ^ m),
                     __uint_as_float(__float_as_uint(x.im) ^ m)};
}
template <>
__device__ __forceinline__ cx<double> negate_if(cx<double> x, uint32_t odd) {
    const uint32_t m = odd << 31;
    const double re = __hiloint2double(__double2hiint(x.re) ^ int(m), __double2loint(x.re));
    const double im = __hiloint2double(__double2hiint(x.im) ^ int(m), __double2loint(x.im));
    return cx<double>{re, im};
}

template <typename R, int RB>
__device__ __forceinline__ void sign(cx<R> *v, const RtOp &op, const Tabs &tb, uint64_t base) {
    constexpr int E = 1 << RB;
    const uint32_t L = terms_live(op, tb, base);
#pragma unroll
    for (int e = 0; e < E; ++e)
        v[e] = negate_if(v[e], uint32_t(__builtin_popcount(L & op.w[32 + e])) & 1u);
}

template <typename R, int RB>
__device__ __forceinline__ void terms(cx<R> *v, const RtOp &op, const Tabs &tb, uint64_t base) {
    constexpr int E = 1 << RB;
    const uint32_t L = terms_live(op, tb, base);
    const int nt = op.nt;
    for (int k = 0; k < nt; ++k) {
        const cx<R> p = ldu<R>(op.u, k);
#pragma unroll
        for (int e = 0; e < E; ++e)
            v[e] = csel((L & op.w[32 + e]) >> k & 1u, cmul(p, v[e]), v[e]);
    }
}

// the thread's phase factor of a fan: its wave entry, the windows of the
// tile's out-of-tile bits (uniform) and its lane entry
template <typename R>
__device__ __forceinline__ cx<R> fan_factor(const RtOp &op, const Tabs &tb, uint64_t base) {
    cx<R> k = ldu<R>(op.ph, int(tb.wave));
    const int nw = op.b;
#pragma unroll
    for (int j = 0; j < kRtWindows; ++j)
        if (j < nw)   // uniform
            k = cmul(k, ldu<R>(op.ph, 8 + 8 * j + int((base >> op.hw[j]) & 7)));
    return cmul(k, reinterpret_cast<const cx<R> *>(tb.ltab + op.w[0])[tb.lane]);
}

// the elements with register bit S set take f times their element factor
template <typename R, int RB, int S>
__device__ __forceinline__ void fan_slot(cx<R> *v, const RtOp &op, cx<R> f) {
    constexpr int E = 1 << RB;
#pragma unroll
    for (int e = 0; e < E; ++e)
        if ((e >> S) & 1) v[e] = cmul(cmul(f, ldu<R>(op.u, e)), v[e]);
}

// fan_slot when the element factor depends only on the register bits above
// slot S (u[e] equals u at e with the bits below S cleared): one product
// with f per distinct factor
template <typename R, int RB, int S>
__device__ __forceinline__ void fan_slot_upper(cx<R> *v, const RtOp &op, cx<R> f) {
    constexpr int H = 1 << (RB - 1 - S);   // values of the bits above S
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int e1 = (h << (S + 1)) | (1 << S);
        const cx<R> g = cmul(f, ldu<R>(op.u, e1));
#pragma unroll
        for (int lo = 0; lo < (1 << S); ++lo) v[e1 | lo] = cmul(g, v[e1 | lo]);
    }
}

// a fan whose target is thread bit a: every element of the threads that
// have it set
template <typename R, int RB>
__device__ __forceinline__ void fan_thread(cx<R> *v, const RtOp &op, const Tabs &tb, uint64_t base) {
    constexpr int E = 1 << RB;
    const cx<R> f = fan_factor<R>(op, tb, base);
    if (((tb.lane | (tb.wave << 6)) >> op.a) & 1u) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cmul(cmul(f, ldu<R>(op.u, e)), v[e]);
    }
}

template <typename R, int RB, int S>
__device__ __forceinline__ void xgate_slot(cx<R> *v, uint32_t rm, uint32_t rv, bool tc) {
    constexpr int E = 1 << RB;
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
        if (e0 & (1 << S)) continue;
        const bool c = tc && (uint32_t(e0) & rm) == rv;   // no branch per pair
        const int e1 = e0 | (1 << S);
        const cx<R> a = v[e0], b = v[e1];
        v[e0] = csel(c, b, a);
        v[e1] = csel(c, a, b);
    }
}


// Exchange through LDS: every thread writes its elements at their slots
// under the old layout, then reads the elements of the new layout.  The
// first barrier keeps the writes behind every read of the previous
// exchange.  Threads past the tile (act false) only take the barriers.  An
// exchange that keeps every wavefront's bits (op.b, set by the host only
// behind an earlier exchange of the same tile) needs neither barrier: each
// wavefront then writes and reads back only the slots it read last.
template <typename R, int RB>
__device__ __forceinline__ void remap(cx<R> *v, cx<R> *lds, const RtOp &op, uint32_t tid, bool act) {
    constexpr int E = 1 << RB;
    constexpr int EB = swz_bits<R>();
    uint32_t t_old = 0, t_new = 0;
#pragma unroll
    for (int k = 0; k < kRtMaxTB; ++k) {
        const uint32_t bit = (tid >> k) & 1u;
        t_old |= bit << op.w[32 + k];
        t_new |= bit << op.w[48 + k];
    }
    t_old = rt_swizzle<EB>(t_old);
    t_new = rt_swizzle<EB>(t_new);
    const bool waves_kept = op.b != 0;   // uniform: the exchange stays inside each wavefront
    if (!waves_kept) __syncthreads();
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) lds[t_old ^ op.w[16 + e]] = v[e];
    }
    if (waves_kept) {   // one wavefront's LDS operations complete in order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[t_new ^ op.w[e]];
    }
}

// remap of both vectors of the backward pass: the slot offsets once, then
// one exchange after the other through the same LDS tile
template <typename R, int RB>
__device__ __forceinline__ void remap2(cx<R> *vp, cx<R> *vl, cx<R> *lds, const RtOp &op, uint32_t tid,
                                       bool act) {
    constexpr int E = 1 << RB;
    constexpr int EB = swz_bits<R>();
    uint32_t t_old = 0, t_new = 0;
#pragma unroll
    for (int k = 0; k < kRtMaxTB; ++k) {
        const uint32_t bit = (tid >> k) & 1u;
        t_old |= bit << op.w[32 + k];
        t_new |= bit << op.w[48 + k];
    }
    t_old = rt_swizzle<EB>(t_old);
    t_new = rt_swizzle<EB>(t_new);
    // op.b: the exchange keeps every wavefront's bits (see remap), so each
    // wavefront only ever touches its own LDS slots and in-order LDS
    // operations replace the barriers
    const bool waves_kept = op.b != 0;
    auto order = [&]() {
        if (waves_kept) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        cx<R> *x = v ? vl : vp;
        order();
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) lds[t_old ^ op.w[16 + e]] = x[e];
        }
        order();
        if (act) {
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = lds[t_new ^ op.w[e]];
        }
    }
}

// Run ops[0 .. n_ops) on the tile at `base` held in v.  The op code is
// kind * 8 + register slot (rt_code), so one flat switch picks the code
// for the op and its slot: one merge of the element registers per op
// (nested switches made the compiler copy all of them at every level).
#define QC_RT_SLOT_CASES(KIND, STMT)                                    \
    case rt_code(KIND, 0): { constexpr int S = 0; STMT; } break;        \
    case rt_code(KIND, 1): if constexpr (RB > 1) { constexpr int S = 1; STMT; } break; \
    case rt_code(KIND, 2): if constexpr (RB > 2) { constexpr int S = 2; STMT; } break; \
    case rt_code(KIND, 3): if constexpr (RB > 3) { constexpr int S = 3; STMT; } break;

// two Hadamard + fan steps (RT_HFAN2): slot A with op's fan, slot B with the
// next op's
#define QC_RT_HFAN2_CASE(A, B)                                                      \
    case rt_hfan2_code(A, B):                                                       \
        if constexpr (A < RB && B < RB && A != B) {                                 \
            h_slot<R, RB, A>(v);                                                    \
            fan_slot<R, RB, A>(v, op, fan_factor<R>(op, tb, base));                 \
            const RtOp &op2 = ops[o + 1];                                           \
            h_slot<R, RB, B>(v);                                                    \
            fan_slot<R, RB, B>(v, op2, fan_factor<R>(op2, tb, base));               \
        }                                                                           \
        ++o;                                                                        \
        break;

template <typename R, int RB>
__device__ __forceinline__ void run_ops(cx<R> *v, cx<R> *lds, uint64_t base, uint32_t tid, bool act,
                               const RtOp *__restrict__ ops, int n_ops, const Tabs &tb) {
    constexpr int E = 1 << RB;
    for (int o = 0; o < n_ops; ++o) {
        const RtOp &op = ops[o];
        const int code = op.kind;
        // thread condition and the tile's out-of-tile condition, folded into
        // the selects of the conditioned kinds (no branch around the op, so
        // every path through the loop body changes the registers in place)
        const bool tc = (tid & op.tm) == op.tv && (base & op.hm) == op.hv;
        switch (code) {
            QC_RT_SLOT_CASES(RT_U1, (u1_slot<R, RB, S, false, false>(v, op, tc)))
            QC_RT_SLOT_CASES(RT_U1C, (u1_slot<R, RB, S, false, true>(v, op, tc)))
            QC_RT_SLOT_CASES(RT_U1R, (u1_slot<R, RB, S, true, false>(v, op, tc)))
            QC_RT_SLOT_CASES(RT_U1RC, (u1_slot<R, RB, S, true, true>(v, op, tc)))
            QC_RT_SLOT_CASES(RT_H, (h_slot<R, RB, S>(v)))
            QC_RT_SLOT_CASES(RT_DIAG1, (diag1_slot<R, RB, S>(v, ldu<R>(op.u, 0), ldu<R>(op.u, 1), op.b != 0)))
            QC_RT_SLOT_CASES(RT_FAN, (fan_slot<R, RB, S>(v, op, fan_factor<R>(op, tb, base))))
            QC_RT_SLOT_CASES(RT_HFAN, (h_slot<R, RB, S>(v), fan_slot<R, RB, S>(v, op, fan_factor<R>(op, tb, base))))
            QC_RT_HFAN2_CASE(0, 1) QC_RT_HFAN2_CASE(0, 2) QC_RT_HFAN2_CASE(0, 3)
            QC_RT_HFAN2_CASE(1, 0) QC_RT_HFAN2_CASE(1, 2) QC_RT_HFAN2_CASE(1, 3)
            QC_RT_HFAN2_CASE(2, 0) QC_RT_HFAN2_CASE(2, 1) QC_RT_HFAN2_CASE(2, 3)
            QC_RT_HFAN2_CASE(3, 0) QC_RT_HFAN2_CASE(3, 1) QC_RT_HFAN2_CASE(3, 2)
        case rt_code(RT_U1X4, 0):
            if constexpr (RB >= 4) {
                u1_slot<R, RB, 0, false, false>(v, op, true);
                u1_slot<R, RB, 1, false, false>(v, ops[o + 1], true);
                u1_slot<R, RB, 2, false, false>(v, ops[o + 2], true);
                u1_slot<R, RB, 3, false, false>(v, ops[o + 3], true);
            }
            o += 3;
            break;
        case rt_code(RT_U1X4X, 0):
            if constexpr (RB >= 4) {
                u1_slot<R, RB, 0, false, false>(v, op, true);
                u1_slot<R, RB, 1, false, false>(v, ops[o + 1], true);
                u1_slot<R, RB, 2, false, false>(v, ops[o + 2], true);
                u1_slot<R, RB, 3, false, false>(v, ops[o + 3], true);
                remap<R, RB>(v, lds, ops[o + 4], tid, act);
            }
            o += 4;
            break;
        case rt_code(RT_U1X3X, 0):
            if constexpr (RB == 3) {   // the host emits it for 8-register programs only
                u1_slot<R, RB, 0, false, false>(v, op, true);
                u1_slot<R, RB, 1, false, false>(v, ops[o + 1], true);
                u1_slot<R, RB, 2, false, false>(v, ops[o + 2], true);
                remap<R, RB>(v, lds, ops[o + 3], tid, act);
            }
            o += 3;
            break;
        case rt_code(RT_U1X3, 0):
            if constexpr (RB >= 3) {
                u1_slot<R, RB, 0, false, false>(v, op, true);
                u1_slot<R, RB, 1, false, false>(v, ops[o + 1], true);
                u1_slot<R, RB, 2, false, false>(v, ops[o + 2], true);
            }
            o += 2;
            break;
        case rt_code(RT_HFAN4U, 0):
            if constexpr (RB == 4) {
                h_slot<R, RB, 0>(v);
                fan_slot_upper<R, RB, 0>(v, op, fan_factor<R>(op, tb, base));
                h_slot<R, RB, 1>(v);
                fan_slot_upper<R, RB, 1>(v, ops[o + 1], fan_factor<R>(ops[o + 1], tb, base));
                h_slot<R, RB, 2>(v);
                fan_slot_upper<R, RB, 2>(v, ops[o + 2], fan_factor<R>(ops[o + 2], tb, base));
                h_slot<R, RB, 3>(v);
                fan_slot_upper<R, RB, 3>(v, ops[o + 3], fan_factor<R>(ops[o + 3], tb, base));
            }
            o += 3;
            break;
        case rt_code(RT_HFAN4, 0):
            if constexpr (RB >= 4) {
                h_slot<R, RB, 0>(v);
                fan_slot<R, RB, 0>(v, op, fan_factor<R>(op, tb, base));
                h_slot<R, RB, 1>(v);
                fan_slot<R, RB, 1>(v, ops[o + 1], fan_factor<R>(ops[o + 1], tb, base));
                h_slot<R, RB, 2>(v);
                fan_slot<R, RB, 2>(v, ops[o + 2], fan_factor<R>(ops[o + 2], tb, base));
                h_slot<R, RB, 3>(v);
                fan_slot<R, RB, 3>(v, ops[o + 3], fan_factor<R>(ops[o + 3], tb, base));
            }
            o += 3;
            break;
            QC_RT_SLOT_CASES(RT_CX, (xgate_slot<R, RB, S>(v, op.rm, op.rv, tc)))
        case rt_code(RT_DIAG1, kRtThreadSlot): diag1_thread<R, RB>(v, op, tid); break;
        case rt_code(RT_FAN, kRtThreadSlot): fan_thread<R, RB>(v, op, tb, base); break;
        case rt_code(RT_U2, 0): u2<R, RB, false>(v, op, tc); break;
        case rt_code(RT_U2, 1): u2<R, RB, true>(v, op, tc); break;
        case rt_code(RT_SIGN, 0): sign<R, RB>(v, op, tb, base); break;
        case rt_code(RT_TERMS, 0): terms<R, RB>(v, op, tb, base); break;
        case rt_code(RT_REMAP, 0): remap<R, RB>(v, lds, op, tid, act); break;
        case rt_code(RT_SCALE, 0): {
            const R sc = rt_vals<R>(op.u)[0];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cx<R>{v[e].re * sc, v[e].im * sc};
        } break;
        default: __builtin_unreachable();   // the host emits only the codes above
        }
    }
}

// ---- adjoint backward: the same ops on two vectors, plus gradient steps

#define QC_RT_SLOT_CASES2(KIND, STMT)                                   \
    case rt_code(KIND, 0): { constexpr int S = 0; { cx<R> *V = vp; STMT; } { cx<R> *V = vl; STMT; } } break; \
    case rt_code(KIND, 1): if constexpr (RB > 1) { constexpr int S = 1; { cx<R> *V = vp; STMT; } { cx<R> *V = vl; STMT; } } break; \
    case rt_code(KIND, 2): if constexpr (RB > 2) { constexpr int S = 2; { cx<R> *V = vp; STMT; } { cx<R> *V = vl; STMT; } } break; \
    case rt_code(KIND, 3): if constexpr (RB > 3) { constexpr int S = 3; { cx<R> *V = vp; STMT; } { cx<R> *V = vl; STMT; } } break;

// Im <lam|G|phi> over the pair (phi0, phi1), (lam0, lam1) of one register
// bit for generator G (1 = X, 2 = Y, 3 = Z), in the state's precision
template <typename R>
__device__ __forceinline__ R grad_pair_rt(cx<R> f0, cx<R> f1, cx<R> l0, cx<R> l1, int gen) {
    if (gen == 3) return (l0.re * f0.im - l0.im * f0.re) - (l1.re * f1.im - l1.im * f1.re);
    if (gen == 1) return (l0.re * f1.im - l0.im * f1.re) + (l1.re * f0.im - l1.im * f0.re);
    return -(l0.re * f1.re + l0.im * f1.im) + (l1.re * f0.re + l1.im * f0.im);
}

// the one-qubit matrix (MODE 0 none, 1 general, 2 real, 3 diagonal) on a pair
template <typename R, int MODE>
__device__ __forceinline__ void apply_mode(cx<R> &a0, cx<R> &a1, const cx<R> *u) {
    constexpr int mode = MODE;
    if (mode == 1) {
        const cx<R> z{R(0), R(0)};
        const cx<R> b0 = cfma(u[1], a1, cfma(u[0], a0, z));
        a1 = cfma(u[3], a1, cfma(u[2], a0, z));
        a0 = b0;
    } else if (mode == 2) {
        const cx<R> b0{u[0].re * a0.re + u[1].re * a1.re, u[0].re * a0.im + u[1].re * a1.im};
        a1 = cx<R>{u[2].re * a0.re + u[3].re * a1.re, u[2].re * a0.im + u[3].re * a1.im};
        a0 = b0;
    } else if (mode == 3) {
        a0 = cmul(u[0], a0);
        a1 = cmul(u[3], a1);
    }
}

// add this wavefront's sum of v into its column of gradient slot `slot`
// (each wavefront owns one column: the additions keep a fixed order); the
// sum runs on DPP and permlane exchanges, no LDS round trips
__device__ __forceinline__ void grad_add(double *acc, int slot, uint32_t wave, double v) {
    v = lanes::wave_sum(v);
    if ((threadIdx.x & 63u) == 0) acc[slot * 8 + int(wave)] += v;
}

// partial of generator gen on slot S, then the matrix on both vectors;
// FP64 accumulation of the pair terms
template <typename R, int RB, int S, int MODE>
__device__ __forceinline__ double grad_slot(cx<R> *vp, cx<R> *vl, int gen, const cx<R> *u) {
    constexpr int E = 1 << RB;
    double acc = 0.0;
#pragma unroll
    for (int e0 = 0; e0 < E; ++e0) {
        if (e0 & (1 << S)) continue;
        const int e1 = e0 | (1 << S);
        acc += double(grad_pair_rt<R>(vp[e0], vp[e1], vl[e0], vl[e1], gen));
        apply_mode<R, MODE>(vp[e0], vp[e1], u);
        apply_mode<R, MODE>(vl[e0], vl[e1], u);
    }
    return acc;
}

// a gradient step of MODE on slot S (two for RT_GRAD2)
template <typename R, int RB, int S, int MODE>
__device__ __forceinline__ void grad_op(cx<R> *vp, cx<R> *vl, double *gacc, const RtOp &op, uint32_t wave) {
    cx<R> u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = ldu<R>(op.u, i);
    if (MODE == 4) {   // RT_GRAD2: diagonal step, then real step
        grad_add(gacc, int(op.w[0]), wave, grad_slot<R, RB, S, 3>(vp, vl, op.b & 15, u));
        cx<R> w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = ldu<R>(op.ph, i);
        grad_add(gacc, int(op.w[1]), wave, grad_slot<R, RB, S, 2>(vp, vl, op.b >> 4, w));
    } else {
        grad_add(gacc, int(op.w[0]), wave, grad_slot<R, RB, S, MODE>(vp, vl, op.b, u));
    }
}

// RT_SIGN on both vectors
template <typename R, int RB>
__device__ __forceinline__ void sign2(cx<R> *vp, cx<R> *vl, const RtOp &op, const Tabs &tb, uint64_t base) {
    const uint32_t L = terms_live(op, tb, base);
#pragma unroll
    for (int e = 0; e < (1 << RB); ++e) {
        const uint32_t odd = uint32_t(__builtin_popcount(L & op.w[32 + e])) & 1u;
        vp[e] = negate_if(vp[e], odd);
        vl[e] = negate_if(vl[e], odd);
    }
}

// RT_DGRAD (see qc_internal.h): the block's gradients from the vectors at
// its start, then the product of its inverse rotations on both
template <typename R, int RB>
__device__ __forceinline__ void dgrad(cx<R> *vp, cx<R> *vl, double *gacc, const RtOp &op, const Tabs &tb,
                                      uint64_t base, uint32_t tid) {
    constexpr int E = 1 << RB;
    double T = 0.0, D[RB];
#pragma unroll
    for (int s = 0; s < RB; ++s) D[s] = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double p = double(vl[e].re * vp[e].im - vl[e].im * vp[e].re);
        T += p;
#pragma unroll
        for (int s = 0; s < RB; ++s) D[s] += ((e >> s) & 1) ? -p : p;
    }
    const int nt = op.nt;
    for (int i = 0; i < nt; ++i) {   // uniform
        const uint32_t ent = op.w[1 + i], loc = ent & 0xffu;
        double v;
        if (loc < 8) {
            v = D[0];
#pragma unroll
            for (int s = 1; s < RB; ++s) v = loc == uint32_t(s) ? D[s] : v;
        } else if (loc < 32) {
            v = ((tid >> (loc - 8)) & 1u) ? -T : T;
        } else {
            v = ((base >> (loc - 32)) & 1u) ? -T : T;
        }
        grad_add(gacc, int(ent >> 8), tb.wave, v);
    }
    const cx<R> K = fan_factor<R>(op, tb, base);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const cx<R> f = cmul(K, ldu<R>(op.u, e));
        vp[e] = cmul(f, vp[e]);
        vl[e] = cmul(f, vl[e]);
    }
}

template <typename R, int RB>
__device__ __forceinline__ void run_ops2(cx<R> *vp, cx<R> *vl, cx<R> *lds, double *gacc, uint64_t base,
                                uint32_t tid, bool act, const RtOp *__restrict__ ops, int n_ops,
                                const Tabs &tb) {
    for (int o = 0; o < n_ops; ++o) {
        const RtOp &op = ops[o];
        const int code = op.kind;
        const bool tc = (tid & op.tm) == op.tv && (base & op.hm) == op.hv;
        switch (code) {
            QC_RT_SLOT_CASES(RT_GRAD0, (grad_op<R, RB, S, 0>(vp, vl, gacc, op, tb.wave)))
            QC_RT_SLOT_CASES(RT_GRAD, (grad_op<R, RB, S, 1>(vp, vl, gacc, op, tb.wave)))
            QC_RT_SLOT_CASES(RT_GRADR, (grad_op<R, RB, S, 2>(vp, vl, gacc, op, tb.wave)))
            QC_RT_SLOT_CASES(RT_GRADD, (grad_op<R, RB, S, 3>(vp, vl, gacc, op, tb.wave)))
            QC_RT_SLOT_CASES(RT_GRAD2, (grad_op<R, RB, S, 4>(vp, vl, gacc, op, tb.wave)))
        case rt_code(RT_GRADR3, 0):
            if constexpr (RB >= 3) {
                grad_op<R, RB, 0, 2>(vp, vl, gacc, op, tb.wave);
                grad_op<R, RB, 1, 2>(vp, vl, gacc, ops[o + 1], tb.wave);
                grad_op<R, RB, 2, 2>(vp, vl, gacc, ops[o + 2], tb.wave);
            }
            o += 2;
            break;
        case rt_code(RT_GRADR3X, 0):
            if constexpr (RB >= 3) {
                grad_op<R, RB, 0, 2>(vp, vl, gacc, op, tb.wave);
                grad_op<R, RB, 1, 2>(vp, vl, gacc, ops[o + 1], tb.wave);
                grad_op<R, RB, 2, 2>(vp, vl, gacc, ops[o + 2], tb.wave);
                remap2<R, RB>(vp, vl, lds, ops[o + 3], tid, act);
            }
            o += 3;
            break;
        case rt_code(RT_GRADR2X, 0):
            if constexpr (RB >= 2) {
                grad_op<R, RB, 0, 2>(vp, vl, gacc, op, tb.wave);
                grad_op<R, RB, 1, 2>(vp, vl, gacc, ops[o + 1], tb.wave);
                remap2<R, RB>(vp, vl, lds, ops[o + 2], tid, act);
            }
            o += 2;
            break;
        case rt_code(RT_GRADR2, 0):
            if constexpr (RB >= 2) {
                grad_op<R, RB, 0, 2>(vp, vl, gacc, op, tb.wave);
                grad_op<R, RB, 1, 2>(vp, vl, gacc, ops[o + 1], tb.wave);
            }
            o += 1;
            break;
            QC_RT_SLOT_CASES2(RT_U1, (u1_slot<R, RB, S, false, false>(V, op, tc)))
            QC_RT_SLOT_CASES2(RT_U1C, (u1_slot<R, RB, S, false, true>(V, op, tc)))
            QC_RT_SLOT_CASES2(RT_U1R, (u1_slot<R, RB, S, true, false>(V, op, tc)))
            QC_RT_SLOT_CASES2(RT_U1RC, (u1_slot<R, RB, S, true, true>(V, op, tc)))
            QC_RT_SLOT_CASES2(RT_DIAG1, (diag1_slot<R, RB, S>(V, ldu<R>(op.u, 0), ldu<R>(op.u, 1), op.b != 0)))
            QC_RT_SLOT_CASES2(RT_CX, (xgate_slot<R, RB, S>(V, op.rm, op.rv, tc)))
        case rt_code(RT_DIAG1, kRtThreadSlot):
            diag1_thread<R, RB>(vp, op, tid);
            diag1_thread<R, RB>(vl, op, tid);
            break;
        case rt_code(RT_U2, 0):
            u2<R, RB, false>(vp, op, tc);
            u2<R, RB, false>(vl, op, tc);
            break;
        case rt_code(RT_U2, 1):
            u2<R, RB, true>(vp, op, tc);
            u2<R, RB, true>(vl, op, tc);
            break;
        case rt_code(RT_SIGN, 0): sign2<R, RB>(vp, vl, op, tb, base); break;
        case rt_code(RT_SIGNDG, 0):
            sign2<R, RB>(vp, vl, op, tb, base);
            dgrad<R, RB>(vp, vl, gacc, ops[o + 1], tb, base, tid);
            o += 1;
            break;
        case rt_code(RT_GRADR2R, 0):
            if constexpr (RB >= 2) {
                grad_op<R, RB, 1, 2>(vp, vl, gacc, op, tb.wave);
                grad_op<R, RB, 0, 2>(vp, vl, gacc, ops[o + 1], tb.wave);
            }
            o += 1;
            break;
        case rt_code(RT_TERMS, 0):
            terms<R, RB>(vp, op, tb, base);
            terms<R, RB>(vl, op, tb, base);
            break;
        case rt_code(RT_REMAP, 0): remap2<R, RB>(vp, vl, lds, op, tid, act); break;
        case rt_code(RT_DGRAD, 0): dgrad<R, RB>(vp, vl, gacc, op, tb, base, tid); break;
        default: __builtin_unreachable();   // the backward programs hold no other codes
        }
    }
}

#undef QC_RT_SLOT_CASES2
#undef QC_RT_HFAN2_CASE
#undef QC_RT_SLOT_CASES

}  // namespace rt
}  // namespace qcx
