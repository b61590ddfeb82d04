// Fused 5-qubit block applied on the FP64 matrix cores of gfx950
// (complex128 states).
//
// Same decomposition as the complex64 kernel: a block of gates fused on the
// host into one 32x32 complex U acts as Y = U X, X = the state viewed as a
// 32 x 2^(n-5) matrix (row t = the value of the 5 block qubits, first
// listed qubit = most significant bit of t; column = the other bits), the
// I_l (x) U' (x) I_r product of QCLAB section 3.2 for a 5-qubit U'.
//
// Work decomposition: a workgroup of 8 wavefronts owns a tile of 32 rows x
// 128 columns (tile bits = the 5 target bits plus the 7 lowest other bits:
// 2^12 amplitudes of 16 bytes, 64 KiB of LDS); wavefront w multiplies
// columns 16w .. 16w + 15.
//
//  1. Global -> registers in memory order, one amplitude (16 bytes) per
//     lane per load (tile element j = tid + 512 s), coalesced.
//  2. Registers -> LDS at the swizzled slot sw(j) = j ^ M(j >> 4), M a
//     4x8 GF(2) matrix chosen on the host so that the 16 columns of one row
//     read by a quarter-wavefront land in 16 distinct 16-byte slots.
//  3. 3M complex product on v_mfma_f64_16x16x4_f64:
//     P1 = Ur Xr, P2 = Ui Xi, P3 = (Ur + Ui)(Xr + Xi), Yr = P1 - P2,
//     Yi = P3 - P1 - P2: per wavefront 2 row blocks x 8 K-steps x 3 = 48.
//  4. Results -> LDS (same swizzle) -> registers in memory order -> global.
// U stays in VGPRs for the whole kernel; tiles come from an atomic counter
// (one per value of the selector bits above the tile, zeroed by the
// operand upload), one tile ahead, as in the complex64 kernel.
//
// Multiplexed blocks: a selector bit among the 7 column bits is given one of
// the column-index bits 5, 6 (which pick the wavefront); a selector bit
// above the tile is fixed per workgroup.
//
// Register layouts of v_mfma_f64_16x16x4_f64 (wave64, measured on gfx950):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, register r holds D[l / 16 + 4 r][l % 16]
#include "qc_internal.h"

#include <algorithm>
#include <random>

#include "../../include/qc.h"

namespace qcx {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));   // one amplitude (re, im)

constexpr int kC = 7;                   // column bits
constexpr int kTileBits = 5 + kC;       // 12
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;   // 512; 8 tile elements per thread

struct Mfma128Args {
    cx<double> *amp;
    const double *a_ops;       // per matrix [3][32][32]: Ur, Ui, Ur + Ui (row = output t)
    unsigned *tickets;         // zeroed tile counters, one per selector value, 64 B apart
    uint64_t n_tiles;          // tiles per value of the selector bits above the tile
    uint64_t off_s[8];         // address offset of tile element 512 s
    uint8_t tile_pos[kTileBits];              // ascending bit positions of the tile bits
    uint8_t ins_pos[kTileBits + kMaxSel];     // ascending tile + high selector positions
    uint8_t sel_pos[kMaxSel];  // selector bits above the tile, most significant first
    uint8_t mat_idx[(1 << kMaxSel) * kWaves];   // matrix of [workgroup value][wavefront]
    int n_ins;
    int n_sel;                 // selector bits above the tile
    uint16_t mcol[8];          // swizzle: XOR values of bits 4..11 of j
    uint16_t col_dep[kC];      // compressed index of column bit i
    uint16_t sw_mem_s[8];      // sw(512 s)
    uint16_t sw_rd_s[8];       // sw(dep_T(4 ks)), K-step ks
    uint16_t sw_out[8];        // sw(dep_T(16 rb + 4 r)), index 4 rb + r
    uint16_t t_lane[4];        // dep_T(k), k = 0..3 (row within a K-step)
};

__device__ __host__ inline uint32_t swz128(uint32_t j, const uint16_t *mcol) {
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        if ((j >> (4 + b)) & 1) m ^= mcol[b];
    return j ^ m;
}

__global__ __launch_bounds__(kThreads) void k_fused_mfma_c128(const Mfma128Args a) {
    __shared__ dbl2 lds[1 << kTileBits];
    __shared__ unsigned ticket_lds;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int l = tid & 63;
    const int kq = l >> 4;    // row within a K-step (B operand) / row group (D)
    const int col = l & 15;   // column within the wavefront's 16

    // selector value of this workgroup and the bits it fixes
    const unsigned sel = blockIdx.x & ((1u << a.n_sel) - 1u);
    uint64_t sel_or = 0;
    for (int j = 0; j < a.n_sel; ++j)
        if ((sel >> (a.n_sel - 1 - j)) & 1u) sel_or |= uint64_t(1) << a.sel_pos[j];
    const double *ops = a.a_ops + size_t(a.mat_idx[sel * kWaves + wave]) * 3072;

    // U operands: A[i][k] = U[16 rb + i][4 ks + k], lane holds i = col, k = kq
    double ar[2][8], ai[2][8], as[2][8];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const int idx = (16 * rb + col) * 32 + 4 * ks + kq;
            ar[rb][ks] = ops[idx];
            ai[rb][ks] = ops[1024 + idx];
            as[rb][ks] = ops[2048 + idx];
        }

    // memory-order constants: this thread moves elements tid + 512 s
    uint64_t off_thr = 0;
#pragma unroll
    for (int b = 0; b < 9; ++b)
        if ((tid >> b) & 1) off_thr |= uint64_t(1) << a.tile_pos[b];
    const uint32_t sw_thr = swz128(uint32_t(tid), a.mcol);
    // operand constants: row k = kq of a K-step, column 16 wave + col
    const int ncol = col + 16 * wave;
    uint32_t cdep = 0;
#pragma unroll
    for (int i = 0; i < kC; ++i)
        if ((ncol >> i) & 1) cdep |= uint32_t(1) << a.col_dep[i];
    const uint32_t sw_l = swz128(cdep | a.t_lane[kq], a.mcol);

    // tile base address from registers (no memory loads inside the loop)
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

    unsigned *const counter = a.tickets + 16 * sel;
    unsigned pending = 0;
    if (tid == 0) ticket_lds = atomicAdd(counter, 1u);
    __syncthreads();
    uint64_t tile = ticket_lds;
    __syncthreads();   // every thread has read it before thread 0 writes the next
    if (tile >= a.n_tiles) return;
    dbl2 g[8];
    uint64_t base = tile_base(tile);
#pragma unroll
    for (int s = 0; s < 8; ++s)
        g[s] = __builtin_nontemporal_load(reinterpret_cast<const dbl2 *>(&a.amp[base + off_thr + a.off_s[s]]));
    if (tid == 0) pending = atomicAdd(counter, 1u);

    for (;;) {
        // 2. stage the tile in LDS; publish the ticket taken one tile ago
        if (tid == 0) ticket_lds = pending;
#pragma unroll
        for (int s = 0; s < 8; ++s) lds[sw_thr ^ a.sw_mem_s[s]] = g[s];
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
                    reinterpret_cast<const dbl2 *>(&a.amp[nbase + off_thr + a.off_s[s]]));
            if (tid == 0) pending = atomicAdd(counter, 1u);
        }
        // 3. 3M products
        double4_t p1[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
        double4_t p2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
        double4_t p3[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
            const dbl2 x = lds[sw_l ^ a.sw_rd_s[ks]];
            const double xs = x.x + x.y;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                p1[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[rb][ks], x.x, p1[rb], 0, 0, 0);
                p2[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[rb][ks], x.y, p2[rb], 0, 0, 0);
                p3[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[rb][ks], xs, p3[rb], 0, 0, 0);
            }
        }
        __syncthreads();
        // 4. results back through LDS in memory order
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dbl2 y;
                y.x = p1[rb][r] - p2[rb][r];
                y.y = p3[rb][r] - p1[rb][r] - p2[rb][r];
                lds[sw_l ^ a.sw_out[4 * rb + r]] = y;
            }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 8; ++s)
            __builtin_nontemporal_store(lds[sw_thr ^ a.sw_mem_s[s]],
                                        reinterpret_cast<dbl2 *>(&a.amp[base + off_thr + a.off_s[s]]));
        if (!more) break;
        __syncthreads();
        tile = next;
        base = nbase;
    }
}

// ---- host-side geometry ------------------------------------------------------

// GF(2) rank of up to 8 vectors of 4 bits
int rank4(const uint32_t *cols, int n) {
    uint32_t v[8];
    for (int i = 0; i < n; ++i) v[i] = cols[i];
    int r = 0;
    for (int bit = 0; bit < 4; ++bit) {
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

// Choose M so that the 16 columns x = 0..15 of a row map to 16 distinct
// low-4-bit slots: x -> low4(sw(dep_C(x))) invertible over GF(2).
void choose_swizzle128(const uint16_t *col_dep, uint16_t *mcol) {
    auto ok = [&](const uint16_t *m) {
        uint32_t img[4];
        for (int i = 0; i < 4; ++i) img[i] = swz128(uint32_t(1) << col_dep[i], m) & 15u;
        return rank4(img, 4) == 4;
    };
    uint16_t m[8] = {};
    if (ok(m)) { std::copy(m, m + 8, mcol); return; }
    for (int b = 0; b < 8; ++b) m[b] = uint16_t(b < 4 ? 1u << b : 0u);
    if (ok(m)) { std::copy(m, m + 8, mcol); return; }
    std::mt19937 rng(4321);
    for (int tries = 0; tries < 200000; ++tries) {
        for (int b = 0; b < 8; ++b) m[b] = uint16_t(rng() & 15u);
        if (ok(m)) { std::copy(m, m + 8, mcol); return; }
    }
    for (int b = 0; b < 8; ++b) mcol[b] = 0;  // correct, possibly with conflicts
}

// Fill the launch arguments; false when this geometry does not fit.
bool mfma128_args(int n, const FusedGeom &g, Mfma128Args &a) {
    uint64_t smask = 0;
    for (int j = 0; j < g.n_sel; ++j) smask |= uint64_t(1) << g.sel_pos[j];
    int tpos[5];
    for (int j = 0; j < 5; ++j) tpos[j] = 63 - __builtin_clzll(g.tgt_off[1 << (4 - j)]);
    uint64_t tmask = 0;
    for (int j = 0; j < 5; ++j) tmask |= uint64_t(1) << tpos[j];
    if (tmask & smask) return false;
    // colmask = the 7 lowest non-target bits; selector bits among them take
    // the highest column indices (wavefront bits 5, 6)
    uint64_t colmask = 0;
    int cnt = 0;
    for (int p = 0; p < n && cnt < kC; ++p)
        if (!((tmask >> p) & 1)) {
            colmask |= uint64_t(1) << p;
            ++cnt;
        }
    if (cnt < kC) return false;
    int n_lo = 0;
    for (int j = 0; j < g.n_sel; ++j)
        if ((colmask >> g.sel_pos[j]) & 1) ++n_lo;
    if (n_lo > 2) return false;
    int cpos[kC], nc = 0;
    for (int p = 0; p < n && nc < kC - n_lo; ++p)
        if (((colmask >> p) & 1) && !((smask >> p) & 1)) cpos[nc++] = p;
    int wave_bit[kMaxSel], hi_rank[kMaxSel], lo_seen = 0, hi_seen = 0;
    for (int j = 0; j < g.n_sel; ++j) {
        if ((colmask >> g.sel_pos[j]) & 1) {
            cpos[nc + lo_seen] = g.sel_pos[j];
            wave_bit[j] = kC - n_lo + lo_seen - 4;   // column index bit 4.. = wavefront bit
            hi_rank[j] = -1;
            ++lo_seen;
        } else {
            wave_bit[j] = -1;
            hi_rank[j] = hi_seen;
            a.sel_pos[hi_seen++] = uint8_t(g.sel_pos[j]);
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
    for (int j = 0; j < kC; ++j) tile[5 + j] = cpos[j];
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
    // the 8 loads of a thread move compressed bits 9 .. 11
    for (int s = 0; s < 8; ++s) {
        uint64_t off = 0;
        for (int b = 0; b < 3; ++b)
            if ((s >> b) & 1) off |= uint64_t(1) << tile[9 + b];
        a.off_s[s] = off;
    }
    for (int i = 0; i < kC; ++i) a.col_dep[i] = uint16_t(cidx(cpos[i]));
    auto dep_t = [&](int t) {
        uint32_t j = 0;
        for (int q = 0; q < 5; ++q)
            if ((t >> (4 - q)) & 1) j |= uint32_t(1) << cidx(tpos[q]);
        return j;
    };
    choose_swizzle128(a.col_dep, a.mcol);
    for (int s = 0; s < 8; ++s) a.sw_mem_s[s] = uint16_t(swz128(uint32_t(s) << 9, a.mcol));
    for (int ks = 0; ks < 8; ++ks) a.sw_rd_s[ks] = uint16_t(swz128(dep_t(4 * ks), a.mcol));
    for (int rb = 0; rb < 2; ++rb)
        for (int r = 0; r < 4; ++r)
            a.sw_out[4 * rb + r] = uint16_t(swz128(dep_t(16 * rb + 4 * r), a.mcol));
    for (int k = 0; k < 4; ++k) a.t_lane[k] = uint16_t(dep_t(k));
    return true;
}

int cu_count() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, c = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        cus = c;
    }
    return cus;
}

}  // namespace

bool fused_mfma_c128_fits(int n, const FusedGeom &g) {
    if (g.k != 5 || g.n_sel < 0 || g.n_sel > kMaxSel) return false;
    Mfma128Args a{};
    return mfma128_args(n, g, a);
}

hipError_t launch_fused_mfma_c128(void *amp, int n, const FusedGeom &g, const double *a_dev,
                                  unsigned *tickets, hipStream_t s) {
    if (g.k != 5 || g.n_sel < 0 || g.n_sel > kMaxSel) return hipErrorInvalidValue;
    Mfma128Args a{};
    if (!mfma128_args(n, g, a)) return hipErrorInvalidValue;
    a.amp = static_cast<cx<double> *>(amp);
    a.a_ops = a_dev;
    a.tickets = tickets;
    // one 8-wave workgroup per CU (64 KiB of LDS); a multiple of 2^n_sel
    const uint64_t n_sets = uint64_t(1) << a.n_sel;
    uint64_t grid = a.n_tiles << a.n_sel;
    const uint64_t cap = uint64_t(cu_count());
    if (grid > cap) grid = cap;
    grid &= ~(n_sets - 1);
    if (grid < n_sets) grid = n_sets;
    const int tok = timer_begin("fused_mfma_c128", s);
    hipLaunchKernelGGL(k_fused_mfma_c128, dim3(unsigned(grid)), dim3(kThreads), 0, s, a);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
