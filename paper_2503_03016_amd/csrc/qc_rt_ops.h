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
        if (COND && (uint32_t(e0) & rm) != rv) continue;   // uniform
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
        v[e0] = COND ? csel(tc, x, a) : x;
        v[e1] = COND ? csel(tc, y, b) : y;
    }
}

template <typename R, int RB, bool REAL, bool COND>
__device__ __forceinline__ void u1(cx<R> *v, const RtOp &op, bool tc) {
    switch (op.a) {   // uniform
    case 0: u1_slot<R, RB, 0, REAL, COND>(v, op, tc); break;
    case 1: if constexpr (RB > 1) u1_slot<R, RB, 1, REAL, COND>(v, op, tc); break;
    case 2: if constexpr (RB > 2) u1_slot<R, RB, 2, REAL, COND>(v, op, tc); break;
    case 3: if constexpr (RB > 3) u1_slot<R, RB, 3, REAL, COND>(v, op, tc); break;
    default: break;
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

template <typename R, int RB>
__device__ __forceinline__ void hgate(cx<R> *v, int slot) {
    switch (slot) {
    case 0: h_slot<R, RB, 0>(v); break;
    case 1: if constexpr (RB > 1) h_slot<R, RB, 1>(v); break;
    case 2: if constexpr (RB > 2) h_slot<R, RB, 2>(v); break;
    case 3: if constexpr (RB > 3) h_slot<R, RB, 3>(v); break;
    default: break;
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
        if (COND && (uint32_t(e0) & rm) != rv) continue;
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
        for (int r = 0; r < 4; ++r) v[idx[r]] = COND ? csel(tc, y[r], x[r]) : y[r];
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

// diag(d0, d1) on slot a: a register slot picks per element (uniform), a
// thread slot per thread
template <typename R, int RB>
__device__ __forceinline__ void diag1(cx<R> *v, const RtOp &op, uint32_t tid) {
    constexpr int E = 1 << RB;
    const cx<R> d0 = ldu<R>(op.u, 0), d1 = ldu<R>(op.u, 1);
    const int a = op.a;
    const bool skip0 = op.b != 0;   // d0 == 1
    if (a < RB) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const bool hi = (e >> a) & 1;   // uniform
            if (!hi && skip0) continue;
            v[e] = cmul(hi ? d1 : d0, v[e]);
        }
    } else {
        const bool hi = (tid >> (a - RB)) & 1u;
        const cx<R> d = csel(hi, d1, d0);
        if (skip0 && !hi) return;
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cmul(d, v[e]);
    }
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
    uint32_t L = reinterpret_cast<const uint32_t *>(tb.ltab + op.w[0])[tb.lane];
    L &= reinterpret_cast<const uint32_t *>(tb.gtab + op.w[1])[tb.wave];
    const int nw = op.b;
    for (int j = 0; j < nw; ++j)
        L &= reinterpret_cast<const uint32_t *>(tb.gtab + op.w[2 + j])[(base >> op.hw[j]) & 63];
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
    for (int e = 0; e < E; ++e) {
        const uint32_t re = op.w[32 + e];
        if (!re) continue;   // uniform
        v[e] = negate_if(v[e], uint32_t(__builtin_popcount(L & re)) & 1u);
    }
}

template <typename R, int RB>
__device__ __forceinline__ void terms(cx<R> *v, const RtOp &op, const Tabs &tb, uint64_t base) {
    constexpr int E = 1 << RB;
    const uint32_t L = terms_live(op, tb, base);
    const int nt = op.nt;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t re = op.w[32 + e];
        for (int k = 0; k < nt; ++k) {
            if (!((re >> k) & 1u)) continue;   // uniform
            const cx<R> p = ldu<R>(op.u, k);
            v[e] = csel((L >> k) & 1u, cmul(p, v[e]), v[e]);
        }
    }
}

template <typename R, int RB>
__device__ __forceinline__ void fan(cx<R> *v, const RtOp &op, const Tabs &tb, uint64_t base) {
    constexpr int E = 1 << RB;
    // the factor of the out-of-tile controls (uniform), then the thread part
    cx<R> k = reinterpret_cast<const cx<R> *>(tb.gtab + op.w[1])[tb.wave];
    const int nw = op.b;
    for (int j = 0; j < nw; ++j)
        k = cmul(k, reinterpret_cast<const cx<R> *>(tb.gtab + op.w[2 + j])[(base >> op.hw[j]) & 63]);
    const cx<R> f = cmul(k, reinterpret_cast<const cx<R> *>(tb.ltab + op.w[0])[tb.lane]);
    const int a = op.a;
    if (a < RB) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (!((e >> a) & 1)) continue;   // uniform
            v[e] = cmul(cmul(f, ldu<R>(op.u, e)), v[e]);
        }
    } else {
        // a thread target: the threads with it set (the tables hold 1 for
        // the others would cost a multiply per element; skip them instead)
        if (!((tb.lane | (tb.wave << 6)) >> (a - RB) & 1u)) return;
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

// controlled X on register slot a: swap the pairs whose element condition
// (rm/rv) and thread condition (tm/tv) hold
template <typename R, int RB>
__device__ __forceinline__ void cx_gate(cx<R> *v, const RtOp &op, uint32_t tid) {
    const uint32_t rm = op.rm, rv = op.rv;
    const bool tc = (tid & op.tm) == op.tv;
    switch (op.a) {
    case 0: xgate_slot<R, RB, 0>(v, rm, rv, tc); break;
    case 1: if constexpr (RB > 1) xgate_slot<R, RB, 1>(v, rm, rv, tc); break;
    case 2: if constexpr (RB > 2) xgate_slot<R, RB, 2>(v, rm, rv, tc); break;
    case 3: if constexpr (RB > 3) xgate_slot<R, RB, 3>(v, rm, rv, tc); break;
    default: break;
    }
}

// Exchange through LDS: every thread writes its elements at their slots
// under the old layout, then reads the elements of the new layout.  The
// first barrier keeps the writes behind every read of the previous
// exchange.  Threads past the tile (act false) only take the barriers.
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
    __syncthreads();
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) lds[t_old ^ op.w[16 + e]] = v[e];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds[t_new ^ op.w[e]];
    }
}

// Run ops[0 .. n_ops) on the tile at `base` held in v.
template <typename R, int RB>
__device__ __forceinline__ void run_ops(cx<R> *v, cx<R> *lds, uint64_t base, uint32_t tid, bool act,
                               const RtOp *__restrict__ ops, int n_ops, const Tabs &tb) {
    constexpr int E = 1 << RB;
    for (int o = 0; o < n_ops; ++o) {
        const RtOp &op = ops[o];
        const int kind = op.kind;
        if ((base & op.hm) != op.hv) continue;   // uniform per tile
        switch (kind) {
        case RT_U1:
        case RT_U1R: {
            const bool cond = (op.tm | op.rm) != 0;
            const bool tc = (tid & op.tm) == op.tv;
            if (kind == RT_U1R) {
                if (cond) u1<R, RB, true, true>(v, op, tc);
                else u1<R, RB, true, false>(v, op, tc);
            } else {
                if (cond) u1<R, RB, false, true>(v, op, tc);
                else u1<R, RB, false, false>(v, op, tc);
            }
        } break;
        case RT_H: hgate<R, RB>(v, op.a); break;
        case RT_DIAG1: diag1<R, RB>(v, op, tid); break;
        case RT_U2: {
            const bool tc = (tid & op.tm) == op.tv;
            if ((op.tm | op.rm) != 0) u2<R, RB, true>(v, op, tc);
            else u2<R, RB, false>(v, op, tc);
        } break;
        case RT_SIGN: sign<R, RB>(v, op, tb, base); break;
        case RT_TERMS: terms<R, RB>(v, op, tb, base); break;
        case RT_FAN: fan<R, RB>(v, op, tb, base); break;
        case RT_CX: cx_gate<R, RB>(v, op, tid); break;
        case RT_REMAP: remap<R, RB>(v, lds, op, tid, act); break;
        case RT_SCALE: {
            const R s = rt_vals<R>(op.u)[0];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cx<R>{v[e].re * s, v[e].im * s};
        } break;
        default: break;
        }
    }
}

}  // namespace rt
}  // namespace qcx
