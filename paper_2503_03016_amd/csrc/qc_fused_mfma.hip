// Fused 5-qubit block applied on the FP32 matrix cores of gfx950.
//
// A block of gates fused on the host into one 32x32 complex matrix U acts
// on the state as Y = U X, where X is the state viewed as a 32 x 2^(n-5)
// matrix: row t is the value of the 5 block qubits (first listed qubit =
// most significant bit of t), column c runs over the other bits.  This is
// the I_l (x) U' (x) I_r product of QCLAB section 3.2 for a 5-qubit U'.
//
// Work decomposition: one wavefront owns a tile of 32 rows x 32 columns
// (1024 amplitudes).  Tile bits = the 5 target bits plus the 5 lowest
// other bits; bits 0..4 are therefore always tile bits, so every tile is a
// set of contiguous runs of at least 32 amplitudes (256 bytes) in HBM.
//
//  1. Global -> registers in memory order (lane l, step s: tile element
//     j = l + 64 s), fully coalesced whatever the target positions.
//  2. Registers -> LDS at a swizzled slot sw(j) = j ^ M(j >> 5), with M a
//     5x5 GF(2) matrix chosen on the host so that both the memory-order
//     accesses and the matrix-operand accesses (32 lanes = 32 columns of one
//     row) hit 32 distinct 8-byte slots, i.e. no LDS bank conflicts.
//  3. LDS -> operand registers and 48 v_mfma_f32_32x32x2_f32: the complex
//     product uses the 3M form  P1 = Ur Xr, P2 = Ui Xi,
//     P3 = (Ur + Ui)(Xr + Xi),  Yr = P1 - P2,  Yi = P3 - P1 - P2
//     (3 real 32x32x32 products instead of 4).
//  4. Accumulators -> LDS (same swizzle) -> registers in memory order ->
//     global, again fully coalesced.
// The U operands stay in VGPRs for the whole kernel; the next tile's global
// loads are in flight while the current tile is multiplied.
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

struct MfmaArgs {
    cx<float> *amp;
    const float *a_ops;         // [3][32][32]: Ur, Ui, Ur + Ui (row = output t)
    uint64_t n_tiles;
    uint64_t off_s[16];         // address offset of tile element (s << 6)
    uint8_t tile_pos[10];       // ascending bit positions of the tile bits
    uint16_t mcol[5];           // swizzle matrix columns
    uint16_t col_dep[5];        // compressed index of column bit i
    uint16_t t16, t4;           // compressed index of target local 16 and 4
    uint16_t sw_mem_s[16];      // sw(s << 6)
    uint16_t sw_rd_s[16];       // sw(dep_T(s))
    uint16_t sw_out_s[16];      // sw(dep_T(8 (r/4) + r % 4))
};

__device__ inline uint32_t swz(uint32_t j, const uint16_t *mcol) {
    uint32_t h = j >> 5, m = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
        if ((h >> b) & 1) m ^= mcol[b];
    return j ^ m;
}

constexpr int kWave = 64;

__global__ __launch_bounds__(kWave) void k_fused_mfma_c64(const MfmaArgs a) {
    __shared__ float2 lds[1024];
    const int l = threadIdx.x;
    const int h = l >> 5;
    const int nidx = l & 31;

    // U operands for the 16 K-steps: row m = l % 32, input row t = s + 16 h
    float ar[16], ai[16], as[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int idx = nidx * 32 + s + 16 * h;
        ar[s] = a.a_ops[idx];
        ai[s] = a.a_ops[1024 + idx];
        as[s] = a.a_ops[2048 + idx];
    }

    // per-lane address and LDS slot constants
    uint64_t off_lane = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((l >> b) & 1) off_lane |= uint64_t(1) << a.tile_pos[b];
    uint32_t cdep = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i)
        if ((nidx >> i) & 1) cdep |= uint32_t(1) << a.col_dep[i];
    const uint32_t sw_mem_l = swz(uint32_t(l), a.mcol);
    const uint32_t sw_rd_l = swz(cdep | (h ? a.t16 : 0u), a.mcol);
    const uint32_t sw_out_l = swz(cdep | (h ? a.t4 : 0u), a.mcol);

    uint64_t tile = blockIdx.x;
    if (tile >= a.n_tiles) return;
    float2 g[16];
    uint64_t base = insert_zeros(tile, a.tile_pos, 10);
#pragma unroll
    for (int s = 0; s < 16; ++s)
        g[s] = *reinterpret_cast<const float2 *>(&a.amp[base + off_lane + a.off_s[s]]);

    for (;;) {
        // 2. stage the tile in LDS
#pragma unroll
        for (int s = 0; s < 16; ++s) lds[sw_mem_l ^ a.sw_mem_s[s]] = g[s];
        __syncthreads();
        // prefetch the next tile while this one is multiplied
        const uint64_t next = tile + gridDim.x;
        const bool more = next < a.n_tiles;
        const uint64_t nbase = more ? insert_zeros(next, a.tile_pos, 10) : 0;
        if (more) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                g[s] = *reinterpret_cast<const float2 *>(&a.amp[nbase + off_lane + a.off_s[s]]);
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
        for (int s = 0; s < 16; ++s)
            *reinterpret_cast<float2 *>(&a.amp[base + off_lane + a.off_s[s]]) =
                lds[sw_mem_l ^ a.sw_mem_s[s]];
        if (!more) break;
        __syncthreads();
        tile = next;
        base = nbase;
    }
}

// ---- host-side geometry ------------------------------------------------------

// GF(2) rank of up to 5 column vectors of 5 bits
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

uint32_t apply_m(uint32_t j, const uint16_t *mcol) {
    uint32_t h = j >> 5, m = 0;
    for (int b = 0; b < 5; ++b)
        if ((h >> b) & 1) m ^= mcol[b];
    return j ^ m;
}

// Choose M so that the 32 column slots of a matrix row are 32 distinct
// low-5-bit values after swizzling: the map n -> low5(sw(dep_C(n))) must be
// invertible over GF(2).
void choose_swizzle(const uint16_t *col_dep, uint16_t *mcol) {
    auto ok = [&](const uint16_t *m) {
        uint32_t img[5];
        for (int i = 0; i < 5; ++i) img[i] = apply_m(uint32_t(1) << col_dep[i], m) & 31u;
        return rank5(img, 5) == 5;
    };
    uint16_t m[5] = {0, 0, 0, 0, 0};
    if (ok(m)) { std::copy(m, m + 5, mcol); return; }
    for (int b = 0; b < 5; ++b) m[b] = uint16_t(1u << b);
    if (ok(m)) { std::copy(m, m + 5, mcol); return; }
    std::mt19937 rng(12345);
    for (int tries = 0; tries < 100000; ++tries) {
        for (int b = 0; b < 5; ++b) m[b] = uint16_t(rng() & 31u);
        if (ok(m)) { std::copy(m, m + 5, mcol); return; }
    }
    for (int b = 0; b < 5; ++b) mcol[b] = uint16_t(1u << b);  // unreachable in practice
}

int query_grid_cap() {
    static int cap = 0;
    if (cap == 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        cap = cus * 16;
    }
    return cap;
}

}  // namespace

hipError_t launch_fused_mfma_c64(void *amp, int n, const FusedGeom &g, const float *a_dev,
                                 hipStream_t s) {
    if (g.k != 5 || n < 10) return hipErrorInvalidValue;
    MfmaArgs a{};
    a.amp = static_cast<cx<float> *>(amp);
    a.a_ops = a_dev;
    a.n_tiles = uint64_t(1) << (n - 10);
    // target positions, most significant local bit first
    int tpos[5];
    for (int j = 0; j < 5; ++j) {
        const uint64_t off = g.tgt_off[1 << (4 - j)];
        tpos[j] = 63 - __builtin_clzll(off);
    }
    uint64_t tmask = 0;
    for (int j = 0; j < 5; ++j) tmask |= uint64_t(1) << tpos[j];
    int cpos[5], nc = 0;
    for (int p = 0; p < n && nc < 5; ++p)
        if (!((tmask >> p) & 1)) cpos[nc++] = p;
    int tile[10];
    for (int j = 0; j < 5; ++j) tile[j] = tpos[j];
    for (int j = 0; j < 5; ++j) tile[5 + j] = cpos[j];
    std::sort(tile, tile + 10);
    auto cidx = [&](int p) {
        for (int i = 0; i < 10; ++i)
            if (tile[i] == p) return i;
        return -1;
    };
    for (int i = 0; i < 10; ++i) a.tile_pos[i] = uint8_t(tile[i]);
    for (int sidx = 0; sidx < 16; ++sidx) {
        uint64_t off = 0;
        for (int b = 0; b < 4; ++b)
            if ((sidx >> b) & 1) off |= uint64_t(1) << tile[6 + b];
        a.off_s[sidx] = off;
    }
    for (int i = 0; i < 5; ++i) a.col_dep[i] = uint16_t(cidx(cpos[i]));
    auto dep_t = [&](int t) {
        uint32_t j = 0;
        for (int q = 0; q < 5; ++q)
            if ((t >> (4 - q)) & 1) j |= uint32_t(1) << cidx(tpos[q]);
        return j;
    };
    choose_swizzle(a.col_dep, a.mcol);
    a.t16 = uint16_t(dep_t(16));
    a.t4 = uint16_t(dep_t(4));
    for (int sidx = 0; sidx < 16; ++sidx) {
        a.sw_mem_s[sidx] = uint16_t(apply_m(uint32_t(sidx) << 6, a.mcol));
        a.sw_rd_s[sidx] = uint16_t(apply_m(dep_t(sidx), a.mcol));
        a.sw_out_s[sidx] = uint16_t(apply_m(dep_t(8 * (sidx / 4) + sidx % 4), a.mcol));
    }
    uint64_t grid = a.n_tiles;
    const uint64_t cap = uint64_t(query_grid_cap());
    if (grid > cap) grid = cap;
    const int tok = timer_begin("fused_mfma_c64", s);
    hipLaunchKernelGGL(k_fused_mfma_c64, dim3(unsigned(grid)), dim3(kWave), 0, s, a);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
