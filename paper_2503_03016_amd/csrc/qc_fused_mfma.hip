// Fused 5-qubit block applied on the FP32 matrix cores of gfx950.
//
// A block of gates fused on the host into one 32x32 complex matrix U acts
// on the state as Y = U X, where X is the state viewed as a 32 x 2^(n-5)
// matrix: row t is the value of the 5 block qubits (first listed qubit =
// most significant bit of t), column c runs over the other bits.  This is
// the I_l (x) U' (x) I_r product of QCLAB section 3.2 for a 5-qubit U'.
//
// Work decomposition: a workgroup of W = 2^(C-5) wavefronts owns a tile of
// 32 rows x 2^C columns.  Tile bits = the 5 target bits plus the C lowest
// other bits (C = 8: 2^13 amplitudes, 64 KiB; C = 7 for registers too
// small for that: 2^12, 32 KiB).  The low bits are therefore tile bits, so
// a tile is a set of contiguous runs of at least 2^C amplitudes (2 KiB at
// C = 8) in HBM whatever the target positions.
//
//  1. Global -> registers in memory order, 16 bytes per lane (tile element
//     pair j, j+1 with j = 2 tid + 2 W 64 s), fully coalesced.
//  2. Registers -> LDS at the swizzled slot sw(j) = j ^ M(j >> 5), M a 5xC
//     GF(2) matrix chosen on the host so that the 32 columns of one matrix
//     row read by a half-wavefront land in 32 distinct 8-byte slots (no LDS
//     bank conflicts) wherever the target bits are.
//  3. Wave w multiplies columns 32w..32w+31: LDS -> operand registers, 48
//     v_mfma_f32_32x32x2_f32 in the 3M form  P1 = Ur Xr, P2 = Ui Xi,
//     P3 = (Ur + Ui)(Xr + Xi),  Yr = P1 - P2,  Yi = P3 - P1 - P2.
//  4. Accumulators -> LDS (same swizzle) -> registers in memory order ->
//     global, 16 bytes per lane.
// U stays in VGPRs for the whole kernel; the next tile's loads are in
// flight while the current tile is multiplied.
//
// Tiles are handed out in ascending order from an atomic counter (one per
// value of the selector bits above the tile, zeroed by the upload of the
// operands), one tile ahead of its use: the tiles in flight on all CUs are
// then always a narrow window of consecutive tiles, which streams from HBM
// faster than a fixed tile-to-workgroup assignment whose workgroups drift
// apart.  A workgroup stops at the first ticket past the last tile.
//
// Multiplexed blocks (U_v selected by up to 2 selector bits, the block
// form of a gate controlled from outside it).  A selector bit among the C
// column bits of the tile is given one of the column-index bits 5.. that
// pick the wavefront, so every wavefront still multiplies with one matrix.
// A selector bit above the tile is fixed per workgroup: workgroup b serves
// the value b mod 2^c_hi of those bits only, and its tiles are enumerated
// by inserting zeros at the tile and selector bits.  Each wavefront loads
// its matrix once (mat_idx[workgroup value][wavefront]).
//
// Register layouts of v_mfma_f32_32x32x2_f32 (one block, wave64):
//   A (32x2):  lane l holds A[l % 32][l / 32]
//   B (2x32):  lane l holds B[l / 32][l % 32]
//   D (32x32): lane l, register r holds D[8 (r/4) + 4 (l/32) + r % 4][l % 32]
#include "qc_internal.h"

#include <algorithm>
#include <random>

#include "../../include/qc.h"

namespace qcx {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMaxColBits = 8;
constexpr int kMaxWaves = 1 << (kMaxColBits - 5);

template <int C>
struct MfmaArgs {
    static constexpr int kTileBits = 5 + C;
    cx<float> *amp;
    const float *a_ops;         // per selector value [3][32][32]: Ur, Ui, Ur + Ui (row = output t)
    unsigned *tickets;          // zeroed tile counters, one per selector value, 64 B apart
    uint64_t n_tiles;           // tiles per value of the selector bits above the tile
    uint64_t off_s[8];          // address offset of tile element 2 W 64 s
    uint8_t tile_pos[kTileBits];             // ascending bit positions of the tile bits
    uint8_t ins_pos[kTileBits + kMaxSel];    // ascending tile + high selector bit positions
    uint8_t sel_pos[kMaxSel];   // selector bits above the tile, most significant first
    uint8_t mat_idx[(1 << kMaxSel) * (1 << (C - 5))];   // matrix of [workgroup value][wavefront]
    int n_ins;
    int n_sel;                  // selector bits above the tile
    uint16_t mcol[C];           // swizzle matrix columns (bits 5.. of j)
    uint16_t col_dep[C];        // compressed index of column bit i
    uint16_t t16, t4;           // compressed index of target local 16 and 4
    uint16_t sw_mem_s[8];       // sw(2 W 64 s)
    uint16_t sw_rd_s[16];       // sw(dep_T(s))
    uint16_t sw_out_s[16];      // sw(dep_T(8 (r/4) + r % 4))
};

template <int C>
__device__ __host__ inline uint32_t swz(uint32_t j, const uint16_t *mcol) {
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < C; ++b)
        if ((j >> (5 + b)) & 1) m ^= mcol[b];
    return j ^ m;
}

template <int C>
__global__ __launch_bounds__(64 << (C - 5)) void k_fused_mfma_c64(const MfmaArgs<C> a) {
    constexpr int kTileBits = 5 + C;
    constexpr int kThreads = 64 << (C - 5);
    constexpr int kThrBits = kTileBits - 4;      // compressed bits 1.. moved by the thread index
    __shared__ float2 lds[1 << kTileBits];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int l = tid & 63;
    const int h = l >> 5;
    const int nidx = l & 31;

    // selector value of this workgroup and the bits it fixes
    const unsigned sel = blockIdx.x & ((1u << a.n_sel) - 1u);
    uint64_t sel_or = 0;
    for (int j = 0; j < a.n_sel; ++j)
        if ((sel >> (a.n_sel - 1 - j)) & 1u) sel_or |= uint64_t(1) << a.sel_pos[j];
    const float *ops = a.a_ops + size_t(a.mat_idx[sel * (kThreads / 64) + wave]) * 3072;

    // U operands for the 16 K-steps: row m = l % 32, input row t = s + 16 h
    float ar[16], ai[16], as[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int idx = nidx * 32 + s + 16 * h;
        ar[s] = ops[idx];
        ai[s] = ops[1024 + idx];
        as[s] = ops[2048 + idx];
    }

    // memory-order constants: this thread moves elements 2 tid + 2 kThreads s (+1)
    uint64_t off_thr = 0;
#pragma unroll
    for (int b = 0; b < kThrBits; ++b)
        if ((tid >> b) & 1) off_thr |= uint64_t(1) << a.tile_pos[b + 1];
    const uint32_t sw_thr = swz<C>(uint32_t(2 * tid), a.mcol);
    // operand constants: column n = nidx + 32 wave
    const int ncol = nidx + 32 * wave;
    uint32_t cdep = 0;
#pragma unroll
    for (int i = 0; i < C; ++i)
        if ((ncol >> i) & 1) cdep |= uint32_t(1) << a.col_dep[i];
    const uint32_t sw_rd_l = swz<C>(cdep | (h ? a.t16 : 0u), a.mcol);
    const uint32_t sw_out_l = swz<C>(cdep | (h ? a.t4 : 0u), a.mcol);

    // Tile base address: the tile index with zeros inserted at the tile and
    // high selector positions, held in registers.  (Reading the positions
    // from the argument block inside the loop would be a vector memory load,
    // and waiting for it would also wait for every store still in flight.)
    constexpr int kIns = kTileBits + kMaxSel;
    uint32_t ins[kIns];
#pragma unroll
    for (int j = 0; j < kIns; ++j) ins[j] = a.ins_pos[j];
    const int n_ins = a.n_ins;
    auto tile_base = [&](uint64_t t) {
#pragma unroll
        for (int j = 0; j < kIns; ++j)
            if (j < n_ins) {
                const uint32_t p = ins[j];
                t = ((t >> p) << (p + 1)) | (t & ((uint64_t(1) << p) - 1));
            }
        return t | sel_or;
    };

    // tile tickets: thread 0 takes them, LDS broadcasts them
    __shared__ unsigned ticket_lds;
    unsigned *const counter = a.tickets + 16 * sel;
    unsigned pending = 0;
    if (tid == 0) ticket_lds = atomicAdd(counter, 1u);
    __syncthreads();
    uint64_t tile = ticket_lds;
    __syncthreads();   // every thread has read it before thread 0 writes the next
    if (tile >= a.n_tiles) return;
    floatx4 g[8];
    uint64_t base = tile_base(tile);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        g[s] = __builtin_nontemporal_load(
            reinterpret_cast<const floatx4 *>(&a.amp[base + off_thr + a.off_s[s]]));
    if (tid == 0) pending = atomicAdd(counter, 1u);

    for (;;) {
        // 2. stage the tile in LDS; publish the ticket taken one tile ago
        if (tid == 0) ticket_lds = pending;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint32_t slot = sw_thr ^ a.sw_mem_s[s];
            lds[slot] = make_float2(g[s][0], g[s][1]);
            lds[slot ^ 1u] = make_float2(g[s][2], g[s][3]);
        }
        __syncthreads();
        // prefetch the next tile while this one is multiplied, and take the
        // ticket of the one after it
        const uint64_t next = ticket_lds;
        const bool more = next < a.n_tiles;
        const uint64_t nbase = more ? tile_base(next) : 0;
        if (more) {
#pragma unroll
            for (int s = 0; s < 8; ++s)
                g[s] = __builtin_nontemporal_load(
                    reinterpret_cast<const floatx4 *>(&a.amp[nbase + off_thr + a.off_s[s]]));
            if (tid == 0) pending = atomicAdd(counter, 1u);
        }
        // 3. operands and 3M products
        floatx16 p1 = {0}, p2 = {0}, p3 = {0};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float2 x = lds[sw_rd_l ^ a.sw_rd_s[s]];
            p1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s], x.x, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[s], x.y, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f32_32x32x2f32(as[s], x.x + x.y, p3, 0, 0, 0);
        }
        __syncthreads();
        // 4. results back through LDS in memory order
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            float2 y;
            y.x = p1[r] - p2[r];
            y.y = p3[r] - p1[r] - p2[r];
            lds[sw_out_l ^ a.sw_out_s[r]] = y;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const uint32_t slot = sw_thr ^ a.sw_mem_s[s];
            const float2 y0 = lds[slot], y1 = lds[slot ^ 1u];
            const floatx4 v = {y0.x, y0.y, y1.x, y1.y};
            __builtin_nontemporal_store(v, reinterpret_cast<floatx4 *>(&a.amp[base + off_thr + a.off_s[s]]));
        }
        if (!more) break;
        __syncthreads();
        tile = next;
        base = nbase;
    }
}

// ---- host-side geometry ------------------------------------------------------

// GF(2) rank of up to 8 vectors of 5 bits
int rank5(const uint32_t *cols, int n) {
    uint32_t v[8];
    for (int i = 0; i < n; ++i) v[i] = cols[i];
    int r = 0;
    for (int bit = 0; bit < 5; ++bit) {
        int piv = -1;
        for (int i = r; i < n; ++i)
            if ((v[i] >> bit) & 1) { piv = i; break; }
        if (piv < 0) continue;
        std::swap(v[r], v[piv]);
        for (int i = 0; i < n; ++i)
            if (i != r && ((v[i] >> bit) & 1)) v[i] ^= v[r];
        ++r;
    }
    return r;
}

// Choose M so that the 32 columns n0 = 0..31 of a matrix row map to 32
// distinct low-5-bit slots: n0 -> low5(sw(dep_C(n0))) invertible over GF(2).
template <int C>
void choose_swizzle(const uint16_t *col_dep, uint16_t *mcol) {
    auto ok = [&](const uint16_t *m) {
        uint32_t img[5];
        for (int i = 0; i < 5; ++i) img[i] = swz<C>(uint32_t(1) << col_dep[i], m) & 31u;
        return rank5(img, 5) == 5;
    };
    uint16_t m[C] = {};
    if (ok(m)) { std::copy(m, m + C, mcol); return; }
    for (int b = 0; b < C; ++b) m[b] = uint16_t(b < 5 ? 1u << b : 0u);
    if (ok(m)) { std::copy(m, m + C, mcol); return; }
    std::mt19937 rng(12345);
    for (int tries = 0; tries < 200000; ++tries) {
        for (int b = 0; b < C; ++b) m[b] = uint16_t(rng() & 31u);
        if (ok(m)) { std::copy(m, m + C, mcol); return; }
    }
    for (int b = 0; b < C; ++b) mcol[b] = 0;  // correct, possibly with conflicts
}

int query_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        cus = c;
    }
    return cus;
}

// Fill the launch arguments for column-bit count C; false when the
// register is too small for this tile shape.
template <int C>
bool mfma_args(int n, const FusedGeom &g, MfmaArgs<C> &a) {
    constexpr int kTileBits = 5 + C;
    constexpr int kWaves = 1 << (C - 5);
    uint64_t smask = 0;
    for (int j = 0; j < g.n_sel; ++j) smask |= uint64_t(1) << g.sel_pos[j];
    // target positions, most significant local bit first
    int tpos[5];
    for (int j = 0; j < 5; ++j) {
        const uint64_t off = g.tgt_off[1 << (4 - j)];
        tpos[j] = 63 - __builtin_clzll(off);
    }
    uint64_t tmask = 0;
    for (int j = 0; j < 5; ++j) tmask |= uint64_t(1) << tpos[j];
    if (tmask & smask) return false;
    // colmask = the C lowest non-target bits; selector bits among them take
    // the highest column indices (the wavefront bits), the plain ones keep
    // ascending order below them
    uint64_t colmask = 0;
    int cnt = 0;
    for (int p = 0; p < n && cnt < C; ++p)
        if (!((tmask >> p) & 1)) {
            colmask |= uint64_t(1) << p;
            ++cnt;
        }
    if (cnt < C) return false;
    int n_lo = 0;
    for (int j = 0; j < g.n_sel; ++j)
        if ((colmask >> g.sel_pos[j]) & 1) ++n_lo;
    if (n_lo > C - 5) return false;
    int cpos[kMaxColBits], nc = 0;
    for (int p = 0; p < n && nc < C - n_lo; ++p)
        if (((colmask >> p) & 1) && !((smask >> p) & 1)) cpos[nc++] = p;
    int wave_bit[kMaxSel], hi_rank[kMaxSel], lo_seen = 0, hi_seen = 0;
    for (int j = 0; j < g.n_sel; ++j) {
        if ((colmask >> g.sel_pos[j]) & 1) {
            cpos[nc + lo_seen] = g.sel_pos[j];
            wave_bit[j] = C - n_lo + lo_seen - 5;
            hi_rank[j] = -1;
            ++lo_seen;
        } else {
            wave_bit[j] = -1;
            hi_rank[j] = hi_seen;
            a.sel_pos[hi_seen++] = g.sel_pos[j];
        }
    }
    a.n_sel = hi_seen;
    if (n < kTileBits + a.n_sel) return false;
    a.n_tiles = uint64_t(1) << (n - kTileBits - a.n_sel);
    for (int hv = 0; hv < (1 << a.n_sel); ++hv)
        for (int w = 0; w < kWaves; ++w) {
            int v = 0;
            for (int j = 0; j < g.n_sel; ++j) {
                const int bit = wave_bit[j] >= 0 ? (w >> wave_bit[j]) & 1
                                                 : (hv >> (a.n_sel - 1 - hi_rank[j])) & 1;
                v = 2 * v + bit;
            }
            a.mat_idx[hv * kWaves + w] = uint8_t(v);
        }
    int tile[kTileBits];
    for (int j = 0; j < 5; ++j) tile[j] = tpos[j];
    for (int j = 0; j < C; ++j) tile[5 + j] = cpos[j];
    std::sort(tile, tile + kTileBits);
    auto cidx = [&](int p) {
        for (int i = 0; i < kTileBits; ++i)
            if (tile[i] == p) return i;
        return -1;
    };
    for (int i = 0; i < kTileBits; ++i) a.tile_pos[i] = uint8_t(tile[i]);
    int ins[kTileBits + kMaxSel];
    std::copy(tile, tile + kTileBits, ins);
    for (int j = 0; j < a.n_sel; ++j) ins[kTileBits + j] = a.sel_pos[j];
    a.n_ins = kTileBits + a.n_sel;
    std::sort(ins, ins + a.n_ins);
    for (int i = 0; i < a.n_ins; ++i) a.ins_pos[i] = uint8_t(ins[i]);
    // the 8 loads of a thread move compressed bits kTileBits-3 .. kTileBits-1
    for (int sidx = 0; sidx < 8; ++sidx) {
        uint64_t off = 0;
        for (int b = 0; b < 3; ++b)
            if ((sidx >> b) & 1) off |= uint64_t(1) << tile[kTileBits - 3 + b];
        a.off_s[sidx] = off;
    }
    for (int i = 0; i < C; ++i) a.col_dep[i] = uint16_t(cidx(cpos[i]));
    auto dep_t = [&](int t) {
        uint32_t j = 0;
        for (int q = 0; q < 5; ++q)
            if ((t >> (4 - q)) & 1) j |= uint32_t(1) << cidx(tpos[q]);
        return j;
    };
    choose_swizzle<C>(a.col_dep, a.mcol);
    a.t16 = uint16_t(dep_t(16));
    a.t4 = uint16_t(dep_t(4));
    for (int sidx = 0; sidx < 8; ++sidx)
        a.sw_mem_s[sidx] = uint16_t(swz<C>(uint32_t(sidx) << (kTileBits - 3), a.mcol));
    for (int sidx = 0; sidx < 16; ++sidx) {
        a.sw_rd_s[sidx] = uint16_t(swz<C>(dep_t(sidx), a.mcol));
        a.sw_out_s[sidx] = uint16_t(swz<C>(dep_t(8 * (sidx / 4) + sidx % 4), a.mcol));
    }
    return true;
}

template <int C>
hipError_t launch_c(void *amp, const float *a_dev, unsigned *tickets, MfmaArgs<C> &a,
                    hipStream_t s) {
    constexpr int kWaves = 1 << (C - 5);
    a.amp = static_cast<cx<float> *>(amp);
    a.a_ops = a_dev;
    a.tickets = tickets;
    // the knob counts resident 32 KiB tiles per CU: a 64 KiB workgroup takes two
    int per_cu = knob(QC_KNOB_MFMA_WG_PER_CU) / (kWaves / 4);
    if (per_cu < 1) per_cu = 1;
    // a multiple of 2^n_sel workgroups, so that every value of the selector
    // bits above the tile has the same number of workgroups
    const uint64_t n_sets = uint64_t(1) << a.n_sel;
    uint64_t grid = a.n_tiles << a.n_sel;
    const uint64_t cap = uint64_t(query_cus()) * uint64_t(per_cu);
    if (grid > cap) grid = cap;
    grid &= ~(n_sets - 1);
    if (grid < n_sets) grid = n_sets;
    const int tok = timer_begin("fused_mfma_c64", s);
    hipLaunchKernelGGL((k_fused_mfma_c64<C>), dim3(unsigned(grid)), dim3(64 * kWaves), 0, s, a);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused_mfma_c64(void *amp, int n, const FusedGeom &g, const float *a_dev,
                                 unsigned *tickets, hipStream_t s) {
    if (g.k != 5 || g.n_sel < 0 || g.n_sel > kMaxSel) return hipErrorInvalidValue;
    // 2 KiB contiguous runs (2^13-amplitude tiles) when the register allows,
    // else 1 KiB runs (2^12-amplitude tiles)
    MfmaArgs<8> a8{};
    if (knob(QC_KNOB_MFMA_TILE_BITS) == 13 && mfma_args<8>(n, g, a8))
        return launch_c<8>(amp, a_dev, tickets, a8, s);
    MfmaArgs<7> a7{};
    if (mfma_args<7>(n, g, a7)) return launch_c<7>(amp, a_dev, tickets, a7, s);
    return hipErrorInvalidValue;
}

}  // namespace qcx
