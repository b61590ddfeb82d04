// Qubit permutations: relabelling the qubits of a register moves amplitude
// i to the index whose bits are those of i, moved to new positions.  One
// sweep applies an involution sigma of the bit positions (sigma(sigma(p)) =
// p, e.g. any set of disjoint SWAP gates, section 5.4's two-qubit
// permutation gate); a general permutation is the product of two
// involutions (each cycle is two reflections), so it takes two sweeps.
//
// Tiles: Q = the lowest low_bits positions, their images under sigma, and
// further low positions taken with their images while |Q| <= perm_bits.
// Q is closed under sigma, so sigma maps every tile (the 2^|Q| amplitudes
// sharing the bits outside Q) onto one tile: the tile at sigma(base).  A
// workgroup loads the tile at base and its partner, and writes each one,
// permuted inside, to the other's place; a tile that is its own partner is
// permuted in place.  The low positions keep the HBM runs contiguous.
#include "qc_lanes.h"
#include "qc_tile_ops.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

using tile::kBlock;
// Q grows to kPermBits positions: 2^12 complex64 or 2^11 complex128
// amplitudes (32 KiB, plus padding) per tile, kLowBits of them contiguous
// (512-byte runs in HBM)
constexpr int kPermMaxBits = 12;
__host__ __device__ constexpr int perm_bits(int dtype) { return dtype == QC_C64 ? 12 : 11; }
// tile elements per thread, at most
template <typename R>
constexpr int max_k() { return 1 << (perm_bits(sizeof(R) == 4 ? QC_C64 : QC_C128) - tile::kLoBits); }
__host__ __device__ constexpr int low_bits(int dtype) { return dtype == QC_C64 ? 6 : 5; }

struct PermuteArgs {
    uint64_t n_tiles;
    int m;                          // |Q|
    int n;
    uint32_t pos[kPermMaxBits];     // ascending positions of Q
    uint32_t sigma[QC_MAX_QUBITS];  // destination of each bit position
    // sigma on compressed tile indices, by halves: sigma_Q(j) =
    // sq_lo[j & 63] | sq_hi[j >> 6]
    uint32_t sq_lo[64], sq_hi[64];
};

// LDS slot of tile element j: one padding element after every 32, so that
// the permuted reads (lanes whose elements lie 32 or more apart, e.g. when
// low and high bits trade places) fall in different banks
__device__ inline int padded(int j) { return j + (j >> 5); }

// Write the tile held in registers (v[k] = element threadIdx.x + kBlock k)
// to the tile at `dst`, permuted: element j there is element sigma_Q(j).
// One LDS tile is the exchange buffer; the caller syncs before reusing it.
template <typename R>
__device__ inline void put_permuted(cx<R> *amp, cx<R> *lds, const cx<R> (&v)[max_k<R>()],
                                    uint64_t dst, uint64_t off_lo, uint64_t mask, int T, int K,
                                    const uint32_t (&sq)[max_k<R>()]) {
#pragma unroll
    for (int k = 0; k < max_k<R>(); ++k) {
        const int j = int(threadIdx.x) + k * kBlock;
        if (k < K && j < T) lds[padded(j)] = v[k];
    }
    __syncthreads();
    uint64_t d = 0;
#pragma unroll
    for (int k = 0; k < max_k<R>(); ++k) {
        const int j = int(threadIdx.x) + k * kBlock;
        if (k < K && j < T) amp[dst + off_lo + d] = lds[padded(int(sq[k]))];
        d = tile::next_submask(d, mask);
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_permute_pairs(cx<R> *amp, const PermuteArgs a) {
    extern __shared__ unsigned char smem[];
    const int T = 1 << a.m;
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    const uint64_t off_lo =
        tile::deposit(uint32_t(threadIdx.x) & (T - 1), a.pos, a.m < tile::kLoBits ? a.m : tile::kLoBits);
    const uint64_t mask = tile::hi_mask(a.pos, a.m);
    const int K = T > kBlock ? T >> tile::kLoBits : 1;
    // sigma_Q of this thread's elements, once: the tables sit in the kernel
    // arguments, and a lookup with a per-thread index is a memory load
    uint32_t sq[max_k<R>()];
#pragma unroll
    for (int k = 0; k < max_k<R>(); ++k) {
        const int j = int(threadIdx.x) + k * kBlock;
        sq[k] = k < K && j < T ? (a.sq_lo[j & 63] | a.sq_hi[j >> 6]) : 0u;
    }
    // tile t: its base (the bits of t around Q; a loop of fixed bound, so
    // the positions are read once) and its partner's base sigma(base), the
    // bits moved one per lane (lane p holds sigma(p)) and OR-ed across the
    // wavefront: no chain of dependent scalar loads per tile
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t sig = lane < uint32_t(a.n) ? a.sigma[lane] : 0u;
    auto tile_of = [&](uint64_t t, uint64_t &base, uint64_t &pb) {
        uint64_t g = t;
#pragma unroll
        for (int j = 0; j < kPermMaxBits; ++j)
            if (j < a.m) g = insert_zero(g, int(a.pos[j]));
        base = g;
        const uint64_t mine = lane < uint32_t(a.n) && ((g >> lane) & 1u) ? uint64_t(1) << sig : 0;
        const uint32_t lo = lanes::wave_or(uint32_t(mine)), hi = lanes::wave_or(uint32_t(mine >> 32));
        pb = (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(hi)))) << 32) |
             uint32_t(__builtin_amdgcn_readfirstlane(int(lo)));
    };
    // the next tile from tt on whose partner does not precede it (the
    // workgroup of the partner tile moves both); false past the last
    auto next_pair = [&](uint64_t &tt, uint64_t &base, uint64_t &pb) {
        for (; tt < a.n_tiles; tt += gridDim.x) {   // uniform
            tile_of(tt, base, pb);
            if (pb >= base) return true;
        }
        return false;
    };
    // both tiles' loads in flight before any is waited for
    auto load_pair = [&](cx<R> (&x)[max_k<R>()], cx<R> (&y)[max_k<R>()], uint64_t base, uint64_t pb) {
        const bool pair = pb != base;
        uint64_t d = 0;
#pragma unroll
        for (int k = 0; k < max_k<R>(); ++k) {
            x[k] = k < K ? amp[base + off_lo + d] : cx<R>{R(0), R(0)};
            y[k] = k < K && pair ? amp[pb + off_lo + d] : cx<R>{R(0), R(0)};
            d = tile::next_submask(d, mask);
        }
    };
    uint64_t t = blockIdx.x, base = 0, pb = 0;
    bool have = next_pair(t, base, pb);
    cx<R> va[max_k<R>()], vb[max_k<R>()];
    if (have) load_pair(va, vb, base, pb);
    while (have) {   // uniform
        // the next pair's loads go out before this pair's stores
        uint64_t t2 = t + gridDim.x, base2 = 0, pb2 = 0;
        const bool have2 = next_pair(t2, base2, pb2);
        cx<R> na[max_k<R>()], nb[max_k<R>()];
        if (have2) load_pair(na, nb, base2, pb2);
        // new[sigma(i)] = old[i]: the tile at pb receives the tile at base,
        // permuted by sigma_Q, and the other way round
        put_permuted<R>(amp, lds, va, pb, off_lo, mask, T, K, sq);
        if (pb != base) {
            __syncthreads();
            put_permuted<R>(amp, lds, vb, base, off_lo, mask, T, K, sq);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < max_k<R>(); ++k) {
            va[k] = na[k];
            vb[k] = nb[k];
        }
        t = t2;
        base = base2;
        pb = pb2;
        have = have2;
    }
}

bool is_involution(int n, const uint32_t *sigma) {
    for (int p = 0; p < n; ++p)
        if (sigma[p] >= uint32_t(n) || sigma[sigma[p]] != uint32_t(p)) return false;
    return true;
}

hipError_t permute_involution(void *amp, int dtype, int n, const uint32_t *sigma, hipStream_t s) {
    PermuteArgs a{};
    a.n = n;
    const int max_bits = perm_bits(dtype);
    uint64_t Q = 0;
    const int low = n < low_bits(dtype) ? n : low_bits(dtype);
    for (int p = 0; p < low; ++p)   // at most 2 low_bits <= max_bits positions
        Q |= (uint64_t(1) << p) | (uint64_t(1) << sigma[p]);
    for (int p = low; p < n; ++p) {
        const uint64_t more = (uint64_t(1) << p) | (uint64_t(1) << sigma[p]);
        if (__builtin_popcountll(Q | more) <= max_bits) Q |= more;
    }
    a.m = __builtin_popcountll(Q);
    int cidx[QC_MAX_QUBITS] = {0};
    for (int p = 0, j = 0; p < n; ++p)
        if ((Q >> p) & 1) {
            a.pos[j] = uint32_t(p);
            cidx[p] = j++;
        }
    for (int p = 0; p < n; ++p) a.sigma[p] = sigma[p];
    for (int x = 0; x < 64; ++x)
        for (int c = 0; c < 6; ++c) {
            if (!((x >> c) & 1)) continue;
            if (c < a.m) a.sq_lo[x] |= 1u << cidx[sigma[a.pos[c]]];
            if (c + 6 < a.m) a.sq_hi[x] |= 1u << cidx[sigma[a.pos[c + 6]]];
        }
    a.n_tiles = uint64_t(1) << (n - a.m);
    const size_t elem = dtype == QC_C64 ? 8 : 16;
    const size_t T = size_t(1) << a.m;
    const size_t lds = (T + T / 32) * elem;   // one padded tile
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // an odd grid: the tiles a workgroup visits (t, t + grid, ...) differ in
    // their low bits, so no workgroup keeps drawing the skipped half of the
    // pairs while another draws the pairs
    uint64_t grid = uint64_t(cus) * 4 - 1;
    if (grid > a.n_tiles) grid = a.n_tiles;
    const int tok = timer_begin("permute", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_permute_pairs<float>), dim3(unsigned(grid)), dim3(kBlock), lds, s,
                           static_cast<cx<float> *>(amp), a);
    else
        hipLaunchKernelGGL((k_permute_pairs<double>), dim3(unsigned(grid)), dim3(kBlock), lds, s,
                           static_cast<cx<double> *>(amp), a);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_permute_bits(void *amp, int dtype, int n, const uint32_t *sigma, int *sweeps,
                               hipStream_t s) {
    *sweeps = 0;
    if (n < 1 || n > QC_MAX_QUBITS) return hipErrorInvalidValue;
    bool seen[QC_MAX_QUBITS] = {false};
    bool identity = true;
    for (int p = 0; p < n; ++p) {
        if (sigma[p] >= uint32_t(n) || seen[sigma[p]]) return hipErrorInvalidValue;
        seen[sigma[p]] = true;
        identity = identity && sigma[p] == uint32_t(p);
    }
    if (identity) return hipSuccess;
    if (is_involution(n, sigma)) {
        *sweeps = 1;
        return permute_involution(amp, dtype, n, sigma, s);
    }
    // sigma = B A (A first): on a cycle c_0 -> c_1 -> ... -> c_{k-1} -> c_0,
    // A swaps c_i and c_{-i}, B swaps c_i and c_{1-i} (indices mod k), so
    // c_i -> c_{-i} -> c_{1+i}
    uint32_t A[QC_MAX_QUBITS], B[QC_MAX_QUBITS];
    bool done[QC_MAX_QUBITS] = {false};
    for (int p = 0; p < n; ++p) {
        if (done[p]) continue;
        int cyc[QC_MAX_QUBITS], k = 0;
        for (int q = p; !done[q]; q = int(sigma[q])) {
            done[q] = true;
            cyc[k++] = q;
        }
        for (int i = 0; i < k; ++i) {
            A[cyc[i]] = uint32_t(cyc[(k - i) % k]);
            B[cyc[i]] = uint32_t(cyc[(k + 1 - i) % k]);
        }
    }
    hipError_t e = permute_involution(amp, dtype, n, A, s);
    if (e != hipSuccess) return e;
    e = permute_involution(amp, dtype, n, B, s);
    *sweeps = 2;
    return e;
}

}  // namespace qcx
