// Internal declarations of libqc: device-side helpers and the launchers that
// the C ABI layer (qc_api.cpp) calls.  Nothing here is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace qcx {

// ---- element types ---------------------------------------------------------
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <typename R>
__host__ __device__ inline cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline cx<R> cfma(cx<R> a, cx<R> b, cx<R> acc) {
    // acc + a * b
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}

// Index of group g once zero bits are inserted at the ascending bit
// positions pos[0..m-1] (positions refer to the final index).
//
// Bit-position tables in kernel arguments are 32-bit words: gfx9 has no
// scalar byte load, so a byte table indexed in a loop is read with vector
// loads, and waiting for one of those also waits for every store in flight.
// 32-bit entries at a uniform index are read with scalar loads instead.
__host__ __device__ inline uint64_t insert_zeros(uint64_t g, const uint32_t *pos, int m) {
    for (int j = 0; j < m; ++j) {
        const int p = pos[j];
        const uint64_t lo = g & ((uint64_t(1) << p) - 1);
        g = ((g >> p) << (p + 1)) | lo;
    }
    return g;
}

__host__ __device__ inline uint64_t insert_zero(uint64_t g, int p) {
    const uint64_t lo = g & ((uint64_t(1) << p) - 1);
    return ((g >> p) << (p + 1)) | lo;
}

// ---- limits ----------------------------------------------------------------
constexpr int kMaxPos = 40;        // fixed bit positions of one gate launch
constexpr int kExpectMaxTerms = 32;
constexpr int kReduceBlocks = 1024;  // fixed grid of deterministic reductions

// ---- launch arguments ------------------------------------------------------
// Gate with K target bits and any number of fixed (control) bits.
template <typename R, int K>
struct SmallGateArgs {
    cx<R> *amp;
    uint64_t n_groups;         // 2^(n - K - n_ctrl)
    uint64_t or_bits;          // control values placed at their bit positions
    uint64_t tgt_off[1 << K];  // offset of local index r (bit deposit)
    cx<R> u[(1 << K) * (1 << K)];
    uint32_t pos[kMaxPos];     // ascending positions of targets + controls
    int n_pos;
};

// k-qubit block, optionally multiplexed: with n_sel selector bits the matrix
// applied to a group is U_s, s = the group's values at sel_pos (sel_pos[0]
// = most significant bit of s); the 2^n_sel matrices are stored one after
// the other.
constexpr int kMaxSel = 2;   // U lives in LDS: 4 c128 5-qubit matrices = 64 KiB
struct FusedGeom {
    int k;
    int n_pos;
    uint32_t pos[8];           // ascending target positions
    uint64_t tgt_off[32];      // offset of local index r
    int n_sel;
    uint32_t sel_pos[kMaxSel];  // selector bit positions
};

// One Pauli term of a Hamiltonian on the device: P = i^ph X^x Z^z (masks of
// bit positions), coefficient c.
struct PauliTermDev {
    uint64_t x, z;
    double c;
    int ph;     // number of Y factors mod 4
    int pad;
};

// 2x2 complex matrix in FP64, row-major (entries 0..3 = U00 U01 U10 U11).
struct Mat2d {
    double re[4], im[4];
};

// One gate of an LDS tile run (positions are compressed tile positions).
// TILE_GRAD (adjoint kernel only): accumulate Im <lam|G|phi> for generator
// G (b1: 1 = X, 2 = Y, 3 = Z) on compressed bit b0 into slot `pad`.
// TILE_PHASES: b0 diagonal terms; amplitude i of the tile is multiplied by
// the product of phase t (u[2t], u[2t+1]) over the terms whose conditions
// hold: (i & pm_lo[t]) == pv_lo[t] and (tile_base & pm_hi[t]) == pv_hi[t].
// b1 = the union of the pm_lo masks (at most 8 tile bits).
// TILE_GRAD_APPLY (adjoint kernel only): TILE_GRAD on bit b0, then the
// one-qubit matrix u[0..7] applied to both vectors on the same bit, in one
// pass over the pairs (the partial uses the values before the update).
// TILE_GRAD_APPLY_REAL / _DIAG: the same for a matrix whose imaginary parts
// (inverse RY) or off-diagonal entries (inverse RZ) are all zero.
// TILE_DENSE1_PHASES: the one-qubit matrix u1 on bit b0 (no conditions),
// then the pad diagonal terms of a TILE_PHASES op over the bits b1, in one
// pass over the pairs.
// TILE_FAN: the phases of controlled-phase gates sharing the target bit b0
// (all conditions "= 1"): an amplitude with bit b0 set is multiplied by
// u[2 b0] + i u[2 b0 + 1] (terms on the target alone), by u[2c] + i
// u[2c + 1] for every control bit c of the mask b1 that it has set, and by
// fan_ph[2k] + i fan_ph[2k + 1] for every out-of-tile control k < pad whose
// bit fan_mask[k] the tile has set.  TILE_DENSE1_FAN: the one-qubit matrix
// u1 on bit b0 first, in the same pass over the pairs.
// TILE_GRAD_APPLY2_DIAG_REAL (adjoint kernel only): a TILE_GRAD_APPLY_DIAG
// and a TILE_GRAD_APPLY_REAL op on bit b0 (inverse RZ, then inverse RY) in
// one pass: generator b1 & 15, slot pad & 0xffff, matrix u[0..7] first,
// then generator b1 >> 4, slot pad >> 16, matrix u1.  Each partial uses the
// values before its own matrix.
// TILE_XPERM: b0 controlled-X gates that commute (no target is another's
// target or control) as one permutation of the tile: amplitude i trades
// places with i ^ f(i), f(i) = the OR of 2^x_t[k] over the gates k whose
// controls hold: (i & x_cm[k]) == x_cv[k] and (tile_base & x_hm[k]) ==
// x_hv[k].  The permutation is its own inverse, so one pass of swaps.
// TILE_KRON: b0 = g (2..kKronMax) one-qubit matrices on the distinct
// compressed bits (b1 >> 5j) & 31, j < g, ascending; matrix j is u[8j ..
// 8j + 7].  They commute, so each group of 2^g amplitudes is loaded once and
// the matrices are applied one after another in registers.  No conditions.
enum TileKind {
    TILE_DENSE1 = 0, TILE_DENSE2 = 1, TILE_PHASE = 2, TILE_DIAG1 = 3, TILE_GRAD = 4,
    TILE_PHASES = 5, TILE_GRAD_APPLY = 6, TILE_GRAD_APPLY_REAL = 7, TILE_GRAD_APPLY_DIAG = 8,
    TILE_KRON = 9, TILE_DENSE1_PHASES = 10, TILE_FAN = 11, TILE_DENSE1_FAN = 12,
    TILE_GRAD_APPLY2_DIAG_REAL = 13, TILE_XPERM = 14,
    // backward pass only: a block of commuting diagonal rotations (see
    // RT_DGRAD): in-tile entries on the compressed bits of mask b1 (bit c:
    // the phase of its set value u[2c], u[2c + 1]), out-of-tile entries
    // fan_mask[h] / fan_ph[h] (h < pad), a common factor u1[0], u1[1];
    // gradient slots b0, b0 + 1, ... in that order (in-tile by ascending c)
    TILE_DGRAD = 15
};
constexpr int kXpermTerms = 12;
constexpr int kKronMax = 3;
constexpr int kTileMaxBits = 16;
constexpr int kTilePhaseTerms = 16;
constexpr int kPhaseTableBits = 8;   // in-tile bits a TILE_PHASES op may test
struct TileOp {
    int32_t kind;
    int32_t b0, b1;            // targets (b0 = most significant bit of the local index)
    int32_t pad;
    uint32_t cmask_lo, cval_lo;  // conditions on tile bits (compressed)
    uint64_t cmask_hi, cval_hi;  // conditions on bits outside the tile (global)
    double u[32];              // complex FP64 entries, interleaved
    union {
        struct {               // TILE_PHASES terms
            uint32_t pm_lo[kTilePhaseTerms], pv_lo[kTilePhaseTerms];
            uint64_t pm_hi[kTilePhaseTerms], pv_hi[kTilePhaseTerms];
        };
        struct {               // TILE_FAN out-of-tile controls
            uint64_t fan_mask[kTilePhaseTerms];
            double fan_ph[2 * kTilePhaseTerms];
        };
        struct {               // TILE_XPERM gates
            uint32_t x_cm[kXpermTerms], x_cv[kXpermTerms], x_t[kXpermTerms];
            uint64_t x_hm[kXpermTerms], x_hv[kXpermTerms];
        };
    };
    double u1[8];              // TILE_DENSE1_PHASES / TILE_DENSE1_FAN: the one-qubit matrix
};
static_assert(kTileMaxBits <= 16, "TILE_FAN keeps one phase per tile bit in u");
struct TileArgs {
    uint64_t n_tiles;
    int m;                     // tile bits
    int n_ops;
    uint32_t pos[kTileMaxBits];  // ascending global bit positions of the tile bits
};

// ---- register-resident tile programs ----------------------------------------
//
// A tile of 2^m amplitudes is held in the registers of 2^(m - RB) threads,
// 2^RB amplitudes ("elements") per thread.  A layout assigns every
// compressed tile bit to a slot: slots 0..RB-1 are the bits of the element
// index e, slot RB + k is bit k of the thread index (bits 0..5: lane,
// above: wavefront).  Element e of thread t holds tile element
// j = dep_reg(e) | dep_thr(t).  Gates whose targets sit in register slots
// need no communication at all; diagonal gates need none wherever their
// bits sit; an RT_REMAP op moves bits between register and thread slots
// through LDS (one write and one read per element).  The host schedules the
// remaps (qc_api.cpp) so that every non-diagonal target is a register slot
// when its gate runs.
//
// Conditions of an op: on out-of-tile bits (hm/hv, uniform per tile), on
// thread-index bits (tm/tv, per thread) and on element-index bits (rm/rv,
// uniform per element e).
constexpr int kRtMaxRB = 4;                  // at most 16 elements per thread
constexpr int kRtMaxE = 1 << kRtMaxRB;
constexpr int kRtMaxTB = 9;                  // at most 512 threads per tile
constexpr int kRtTerms = 16;                 // terms of an RT_SIGN / RT_TERMS op
constexpr int kRtFanHi = 24;                 // out-of-tile controls of an RT_FAN op
constexpr int kRtWindows = 8;                // 3-bit out-of-tile windows of an op's tables
// An op's code is rt_code(kind, sub): sub is the register slot for the
// kinds that act on one (kRtThreadSlot: a thread slot, whose thread bit is
// a), 1 for a conditioned RT_U2, else 0.
enum RtKind {
    RT_U1 = 0,      // u[0..7] (2x2) on register slot sub
    RT_U1C = 1,     // the same where the conditions hold
    RT_U1R = 2,     // real 2x2 (imaginary parts 0) on register slot sub
    RT_U1RC = 3,    // the same where the conditions hold
    RT_H = 4,       // (x0 + x1, x0 - x1) on register slot sub (the 1/sqrt2 is deferred to RT_SCALE)
    RT_DIAG1 = 5,   // diag(u[0..1], u[2..3]) on slot sub; b = 1: u[0..1] == 1
    RT_U2 = 6,      // u[0..31] (4x4) on register slots a (msb of the local index) and b
    RT_SIGN = 7,    // -1 where an odd number of the nt terms hold
    RT_TERMS = 8,   // x phase k (u[2k], u[2k+1]) where term k holds, k < nt
    RT_FAN = 9,     // controlled-phase fan on the target slot sub (see below)
    RT_CX = 10,     // X on register slot sub (swap of the pair) where the conditions hold
    RT_REMAP = 11,  // new layout through LDS
    RT_SCALE = 12,  // x u[0] (real) everywhere
    // adjoint backward only (two vectors phi, lam in registers): the
    // partial Im <lam|G|phi> of generator G (b: 1 = X, 2 = Y, 3 = Z) on
    // register slot sub, added to gradient slot w[0], taken before the
    // one-qubit matrix u is applied to both vectors: RT_GRAD0 applies none,
    // RT_GRAD a general one, RT_GRADR a real one, RT_GRADD a diagonal one
    RT_GRAD0 = 13,
    RT_GRAD = 14,
    RT_GRADR = 15,
    RT_GRADD = 16,
    // an RT_GRADD step and an RT_GRADR step on the same slot: generator
    // b & 15, slot w[0], matrix u; then generator b >> 4, slot w[1], matrix ph
    RT_GRAD2 = 17,
    // forward only: RT_H on register slot sub, then the RT_FAN of that
    // target slot (one op, one pass over the registers)
    RT_HFAN = 18,
    // forward only: two RT_HFAN steps on register slots a != b, the first
    // with this op's fan data, the second with the next op's (a data-only
    // op the interpreter skips); code rt_hfan2_code(a, b), kinds 19 and 20
    RT_HFAN2 = 19,
    // backward only: a block of commuting diagonal rotations exp(-i t Z_q / 2)
    // (their inverses).  Every gradient of the block is Im <lam|Z_q|phi> of
    // the vectors at the block's start (diagonal gates commute with each
    // other and with Z_q), so the op takes p = Im(conj(lam) phi) of each
    // element once and sums it with the sign of bit q: entry i (i < nt) is
    // w[1 + i] = loc | slot << 8, loc < 8 a register slot, 8 + k thread bit
    // k, 32 + p global bit p outside the tile.  Then both vectors take the
    // product of the inverses: element factor u[e] times the RT_FAN thread
    // and window factors (w[0], ph, b, hw as for RT_FAN).
    RT_DGRAD = 21,
    // forward only, 16 registers: RT_HFAN steps on register slots 0, 1, 2
    // and 3 in that order, with this op's fan data and the next three ops'
    // (data-only ops the interpreter skips)
    RT_HFAN4 = 22,
    // RT_HFAN4 where the element factor of step k depends only on the
    // register bits of slots above k (the QFT's fans: their in-register
    // controls are the later targets), so step k forms 2^(3-k) products
    RT_HFAN4U = 23,
    // backward only: RT_GRADR steps on register slots 0, 1, 2 (RT_GRADR3)
    // or 0, 1 (RT_GRADR2) in that order, with this op's data and the next
    // ops' (data-only ops the interpreter skips)
    RT_GRADR3 = 24,
    RT_GRADR2 = 25,
    // forward only: unconditioned RT_U1 steps on register slots 0, 1, 2, 3
    // (RT_U1X4) or 0, 1, 2 (RT_U1X3) in that order, with this op's matrix
    // and the next ops' (data-only ops the interpreter skips)
    RT_U1X4 = 26,
    RT_U1X3 = 27,
    // RT_GRADR3 (backward) / RT_U1X4 (forward) followed by the RT_REMAP op
    // that comes after its data ops, in one interpreter step
    RT_GRADR3X = 28,
    RT_U1X4X = 29,
    // the same for RT_GRADR2 and RT_U1X3 (the latter in 8-register programs)
    RT_GRADR2X = 30,
    RT_U1X3X = 31,
    // backward only: RT_GRADR steps on slots 1 then 0; an RT_SIGN op and the
    // RT_DGRAD op behind it
    RT_GRADR2R = 32,
    RT_SIGNDG = 33,
};
constexpr int kRtThreadSlot = 7;
__host__ __device__ constexpr int rt_code(int kind, int sub) { return kind * 8 + sub; }
__host__ __device__ constexpr int rt_hfan2_code(int a, int b) { return RT_HFAN2 * 8 + a * 4 + b; }
// Lookup tables.  Tables indexed by the lane number sit in the program's
// table blob, which is copied to LDS once per workgroup (byte offset w[0]);
// tables indexed by the wavefront number (8 entries) or by a window of 3
// out-of-tile index bits (8 entries, window j at bit hw[j] of the tile
// base, b windows) are stored in the op itself and read with uniform loads.
// RT_SIGN / RT_TERMS: the set L of terms whose thread and tile conditions
// hold is L_lane[lane] & w[8 + wave] & (AND over the windows of
// wt[8j + window value]) (uint32 bit masks); term k then applies to
// element e when bit k of w[32 + e] is set (its condition on the element
// index).
// RT_FAN (sub = target slot; for a register target the factors apply to
// the elements with the target bit set, for a thread target to every
// element of the threads with it set): element e is multiplied by
// u[2e] + i u[2e+1] (the target-only phase and the register-slot controls)
// and by the product of the phases of the controls on thread bits and
// out-of-tile bits: F_lane[lane] (complex lane table), ph entry wave
// (complex index) and ph entry 8 + 8j + window value for every window j
// (values in the state's precision).
// RT_REMAP: the thread part of an element's LDS slot is swz(sum of bit k of
// t << w[32 + k]) before, swz(sum of bit k of t << w[48 + k]) after; the
// element part is w[16 + e] before and w[e] after (both swizzled tile
// indices); see rt_swizzle.
// Matrix entries and phases are stored in the precision of the state
// (float for complex64 programs, double for complex128): u and ph are
// read through rt_u / rt_ph.
struct RtOp {
    int32_t kind, a, b, nt;
    uint32_t tm, tv, rm, rv;
    uint64_t hm, hv;
    double u[32];
    uint32_t w[64];
    uint64_t hw[2 * kRtFanHi];
    double ph[2 * (8 + 8 * kRtWindows)];   // RT_FAN: wave table, then the window tables
    uint32_t wt[8 * kRtWindows];            // RT_SIGN / RT_TERMS window tables
};
// entry i of the op's u (or ph) array in precision R: float programs pack
// their values into the first half of the double array's bytes
template <typename R>
__host__ __device__ inline R *rt_vals(double *a) { return reinterpret_cast<R *>(a); }
template <typename R>
__host__ __device__ inline const R *rt_vals(const double *a) {
    return reinterpret_cast<const R *>(a);
}
static_assert(sizeof(RtOp) % 16 == 0, "ops are read as 16-byte words");

// LDS slot of tile element j for an exchange: XOR of the bank bits with a
// fold of the higher bits (a bijection of [0, 2^m), linear over GF(2), so
// swz(a | b) = swz(a) ^ swz(b) for disjoint a, b).  EB = log2 of the
// elements in one 128-byte row of LDS banks.
template <int EB>
__host__ __device__ inline uint32_t rt_swizzle(uint32_t j) {
    constexpr uint32_t M = (1u << EB) - 1;
    return j ^ (((j >> EB) ^ (j >> (2 * EB)) ^ (j >> (3 * EB))) & M);
}

struct RtArgs {
    uint64_t n_tiles;
    int m;                       // tile bits
    int tb;                      // thread bits (m - RB)
    int n_ops;
    int pad;
    uint32_t pos[kTileMaxBits];  // ascending global positions of the tile bits
    uint32_t ld_thr[kRtMaxTB];   // global position of thread bit k when loading
    uint32_t st_thr[kRtMaxTB];   // ... and when storing
    uint32_t ld_reg[kRtMaxRB];   // global position of element bit i when loading
    uint32_t st_reg[kRtMaxRB];   // ... and when storing
    uint32_t lds_tab_bytes;      // leading bytes of the table blob that go to LDS
    double st_scale;             // factor of every amplitude at the store (1: none)
};

// One Pauli term of a tile pass of the expectation: X bits xc and Z bits zc
// inside the tile (compressed positions), Z bits z_hi outside it (global
// positions), ph = number of Y factors mod 4, xtop = top bit of xc.
struct ExpectTerm {
    uint64_t z_hi;
    uint32_t xc, zc;
    int32_t ph, xtop;
};
constexpr int kExpectTileMaxTerms = 512;   // terms per tile-pass launch
constexpr int kExpectLowBits = 6;          // lowest bits, always tile bits (runs of 64)

// Register-tile expectation passes (qc_expect_tiles.hip): a wavefront owns
// a tile of 2^(6 + kExpRegB) amplitudes, lane k of the index on global bit
// lpos[k], element bit i on rpos[i]; lane l holds elements e = 0..15 at
// base | dep(l, lpos) | dep(e, rpos).  A term P = i^ph X^x Z^z with x inside
// the tile is split over the slots: x = (xl on lanes, xr on elements), the
// Z bits on lanes zl, on elements zr (zsign: bit e set when e & zr has odd
// parity), outside the tile z_hi.  Diagonal terms (x = 0) name the index
// hk of their zr in the launch's list of distinct element masks hval, and
// those with z_hi != 0 the index ck of their (zsign, zl) pair in the
// launch's list of such pairs (ck = -1 when z_hi = 0).
// X terms carry kind = 2 mode + (ph odd): mode i < 4 the element bit i,
// 4 + b lane bit b < 4, 8 any other lane mask.
struct ExpRegTerm {
    uint64_t z_hi;
    uint32_t xl, xr, zl, zsign;
    int32_t ph, hk, ck, kind;
};
constexpr int kExpRegB = 4;            // element bits per lane (16 amplitudes)
constexpr int kExpRegMaxX = 16;        // X terms per launch (register accumulators)
constexpr int kExpRegMaxD = 64;        // diagonal terms per launch (one per lane)
constexpr int kExpRegMaxH = 1 << kExpRegB;
constexpr int kExpRegMaxC = 8;         // (zsign, zl) pairs of diagonal terms with z_hi != 0
struct ExpRegArgs {
    uint64_t n_tiles;                  // wavefront tiles, 2^(n - 6 - kExpRegB)
    uint32_t pos[6 + kExpRegB];        // ascending global positions of the tile bits
    uint32_t lpos[6];
    uint32_t rpos[kExpRegB];
    uint32_t hval[kExpRegMaxH];
    uint32_t hoff[kExpRegMaxH + 1];    // diagonal terms of mask hval[h]: [hoff[h], hoff[h + 1])
    uint32_t csign[kExpRegMaxC];       // pairs (zsign, zl) of the diagonal terms with z_hi != 0
    uint32_t clane[kExpRegMaxC];
    int32_t n_x, n_d, n_h;             // X terms (first in the term array), diagonal terms, masks
    int32_t n_c, n_din;                // pairs; diagonal terms with z_hi = 0
    // the last n_xb X terms refer to the transposed tile (complex64 only):
    // lane bit k on tile bit tl[k], element bit i on tile bit te[i] (tile
    // bit j < 6 is lane bit j, 6 + i element bit i of the loaded layout);
    // in LDS tile index j sits at j + tpad (j >> tsh)
    int32_t n_xb;
    uint32_t tl[6], te[kExpRegB];
    uint32_t tsh, tpad;
};
// LDS bytes per wavefront of a k_expect_reg launch: per-lane slots of the X
// terms and of the (zsign, zl) pairs, then the transposition buffer
__host__ __device__ inline size_t expect_reg_wave_lds(const ExpRegArgs &a, size_t amp_bytes) {
    const size_t tb = a.n_xb > 0 ? (1024 + a.tpad * (1024u >> a.tsh)) * amp_bytes : 0;
    return size_t(a.n_x + a.n_c) * 64 * sizeof(double) + tb;
}

// ---- batched persistent launch: device program ---------------------------
enum BatchFlags { BATCH_INIT = 1, BATCH_STORE = 2 };
struct BatchPhase {
    uint64_t n_tiles;
    int32_t m, op_begin, op_count, term_begin, term_count, flags;
    uint32_t pos[kTileMaxBits];    // ascending global bit positions of the tile bits
};
struct BatchTerm {
    uint64_t z_hi;     // z bits outside the tile (global positions)
    uint32_t xc, zc;   // x and z inside the tile (compressed positions)
    double c;          // coefficient
    int32_t ph;        // number of Y factors mod 4
    int32_t xtop;      // top bit of xc, -1 when xc == 0
};
struct BatchCircuit {
    uint64_t arena_off;   // element offset of the state in the arena
    int32_t n, phase_begin, phase_count, large;
};
constexpr int kBatchGroup = 8;     // workgroups per group
struct BatchJob {
    int32_t kind;                  // 0: bundle of small circuits, 1: one large circuit
    int32_t circ[kBatchGroup];     // circuit per workgroup (bundle) or circ[0]; -1 = none
};
struct BatchArgs {
    const BatchCircuit *circ;
    const BatchPhase *phases;
    const TileOp *ops;
    const BatchTerm *terms;
    const BatchJob *jobs;
    const int32_t *group_jobs;     // CSR over groups (n_groups + 1 entries)
    void *arena;
    double *energy;
    double *partial;               // circuits x G
    unsigned *barrier;             // n_groups counters, then the error flag
    unsigned *error;
    int n_groups;
    int G;
};

// ---- launchers (return hipSuccess or the launch error) ----------------------
hipError_t launch_init(void *amp, int dtype, int n, uint64_t basis, hipStream_t s);
hipError_t launch_copy(void *dst, int dt_dst, const void *src, int dt_src, uint64_t count,
                       hipStream_t s);
hipError_t launch_small_gate(void *amp, int dtype, int n, int k, const int *tpos_msb_first,
                             int n_ctrl, const int *cpos, const int *cval, const double *u,
                             hipStream_t s);
hipError_t launch_phase(void *amp, int dtype, int n, int m, const int *pos, const int *val,
                        double phase_re, double phase_im, hipStream_t s);
hipError_t launch_fused_valu(void *amp, int dtype, int n, const FusedGeom &g,
                             const void *u_dev, hipStream_t s);
// tickets: kMfmaTicketBytes of zeroed device memory private to this launch
constexpr size_t kMfmaTicketBytes = 64 * (1 << kMaxSel);
hipError_t launch_fused_mfma_c64(void *amp, int n, const FusedGeom &g, const float *a_dev,
                                 unsigned *tickets, hipStream_t s);
// complex128 on the FP64 matrix cores: a_dev per matrix [3][32][32] doubles
// (Ur, Ui, Ur + Ui); fused_mfma_c128_fits tells whether a geometry fits
bool fused_mfma_c128_fits(int n, const FusedGeom &g);
hipError_t launch_fused_mfma_c128(void *amp, int n, const FusedGeom &g, const double *a_dev,
                                  unsigned *tickets, hipStream_t s);
hipError_t launch_probs_full(const void *amp, int dtype, int n, const int *perm_pos,
                             bool identity, double *out, hipStream_t s);
// FP64 workspace entries launch_probs_marginal needs for (n, m): 0 when
// every bin is one block that writes its sum straight to the output
size_t probs_marginal_work(int n, int m);
hipError_t launch_probs_marginal(const void *amp, int dtype, int n, int m, const int *pos,
                                 double *out, double *work, size_t work_elems, hipStream_t s);
hipError_t launch_expect_group(const void *amp, int dtype, int n, uint64_t xmask, int hpos,
                               int n_terms, const uint64_t *zmask, const int *phase,
                               double *term_vals, double *work, hipStream_t s);
hipError_t launch_expect_combine(const double *term_vals, const double *coeff_dev, int n_terms,
                                 int per_term, double *out, hipStream_t s);
hipError_t launch_diff(const void *a, int dt_a, const void *b, int dt_b, uint64_t count,
                       double *out, double *work, hipStream_t s);

hipError_t launch_tile_run(void *amp, int dtype, int n, const TileArgs &a, const TileOp *ops_dev,
                           hipStream_t s);
// register bits of the register-resident tile kernel for an element type
// and tile size: complex64 keeps 16 amplitudes per thread; complex128 keeps
// 8 in tiles of up to 2^12 amplitudes (two workgroups per CU) and 16 in the
// wide 2^13-amplitude tiles (a 128 KiB exchange area, one workgroup per CU)
constexpr int kRtWideBits = 13;
constexpr int rt_reg_bits(int dtype, int m) { return dtype == 1 ? 4 : (m >= kRtWideBits ? 4 : 3); }
hipError_t launch_rt_run(void *amp, int dtype, const RtArgs &a, const RtOp *ops_dev,
                         const unsigned char *tabs_dev, hipStream_t s);
// new[sigma(i)] = old[i], sigma moving bit position p to sigma[p] (a
// permutation of 0..n-1, host array); *sweeps receives 0, 1 or 2
hipError_t launch_permute_bits(void *amp, int dtype, int n, const uint32_t *sigma, int *sweeps,
                               hipStream_t s);
// vals[k] = <psi|P_k|psi> for the nt terms of one tile pass; part holds
// nt x grid partials
hipError_t launch_expect_tiles(const void *amp, int dtype, const TileArgs &a,
                               const ExpectTerm *terms_dev, int nt, double *vals, double *part,
                               hipStream_t s);
// vals[k] = <psi|P_k|psi> for the n_x + n_d terms of one register-tile
// launch (X terms first); part holds (n_x + n_d) x grid partials
hipError_t launch_expect_reg(const void *amp, int dtype, const ExpRegArgs &a,
                             const ExpRegTerm *terms_dev, double *vals, double *part,
                             hipStream_t s);
unsigned expect_reg_grid(uint64_t n_tiles);
// lam = sum over the launch's terms of coef[k] P_k psi (the terms in the
// k_expect_reg layout, coefficients in the same order); accumulate: lam +=
hipError_t launch_pauli_reg(const void *psi, void *lam, int dtype, const ExpRegArgs &a,
                            const ExpRegTerm *terms_dev, const double *coef_dev, bool accumulate,
                            hipStream_t s);

hipError_t launch_collapse(void *amp, int dtype, int n, int p, int b, const double *prob,
                           double *prob_out, hipStream_t s);
hipError_t launch_reset(void *amp, int dtype, int n, int p, int b, const double *prob,
                        double *prob_out, hipStream_t s);
// counts[s] (2^m int64, zeroed here) = shots whose index reads s at pos[]
hipError_t launch_count(const int64_t *idx, int shots, int m, const int *pos, int64_t *counts,
                        hipStream_t s);
hipError_t launch_reduced(const void *src, void *dst, int dtype, int n, int m, const int *pos,
                          const int *val, hipStream_t s);
hipError_t launch_sample(const void *amp, int dtype, int n, const double *u, int shots,
                         int64_t *out, double *work, size_t work_elems, hipStream_t s);

int batch_resident_blocks(int dtype, size_t lds_bytes);
hipError_t launch_batch(const BatchArgs &a, int dtype, unsigned grid, size_t lds_bytes,
                        hipStream_t s);

constexpr int kAdjointMaxSlots = 512;   // rotations per adjoint tile run
static_assert(kAdjointMaxSlots <= 65536, "TILE_GRAD_APPLY2 packs two slots in 16 bits each");
unsigned adjoint_tile_grid(uint64_t n_tiles);
// out = H psi (accumulate: out += H psi), one gather per term and amplitude
hipError_t launch_pauli_apply(const void *psi, void *out, int dtype, int n,
                              const PauliTermDev *terms, int nt, bool accumulate, hipStream_t s);
// backward pass on register tiles: both vectors; partial[row][col] as for
// launch_adjoint_tiles (slot_row maps the program's gradient slots to rows)
hipError_t launch_rt_adjoint(void *phi, void *lam, int dtype, const RtArgs &a, const RtOp *ops_dev,
                             const unsigned char *tabs_dev, const int32_t *slot_row_dev,
                             int n_slots, double *partial, unsigned cols, hipStream_t s);
constexpr int kRtAdjSlots = 256;   // gradient slots of one register-tile backward launch
// register bits of the backward kernel (two vectors share the registers)
constexpr int rt_adj_reg_bits(int dtype) { return dtype == 1 ? 3 : 2; }
hipError_t launch_adjoint_tiles(void *phi, void *lam, int dtype, const TileArgs &a,
                                const TileOp *ops_dev, const int32_t *slot_row_dev, int n_slots,
                                double *partial, unsigned cols, hipStream_t s);
hipError_t launch_grad_finalize(const double *partial, int rows, int cols, double *g_op,
                                const int *ptr, const int *idx, int n_params, double *grad,
                                hipStream_t s);

// ---- library services implemented in qc_api.cpp -----------------------------
int knob(int which);   // current value of a QC_KNOB_* launch-shape knob
int timer_begin(const char *name, hipStream_t s);
void timer_end(int token, hipStream_t s);

}  // namespace qcx
