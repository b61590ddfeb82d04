// Batched persistent launch: many circuits of uneven size, each ending in an
// energy <H> = sum_t c_t <psi|P_t|psi>, in ONE kernel launch.
//
// The grid holds only as many workgroups as can be resident at once.  It is
// split into groups of G workgroups (the members of a group are placed on
// the same XCD under round-robin dispatch, so they share one L2).  The host
// assigns every group a list of jobs (longest first, least-loaded group):
//   * a bundle of up to G small circuits: each workgroup runs one circuit
//     alone, entirely inside LDS (init, every gate, the energy) - no HBM
//     traffic for the state at all;
//   * one large circuit: the G workgroups run its phases together.  A phase
//     is a run of gates on one choice of tile bits (as in the tile-run
//     kernel); the tiles of a phase are split over the group, and the group
//     meets at a device-side barrier between phases.
// Barriers are bounded: a workgroup that waits too long sets an error flag
// and moves on, so every workgroup always reaches the end of the kernel.
#include "qc_tile_ops.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

using tile::kBlock;
constexpr int kWaves = kBlock / 64;
constexpr unsigned kSpinLimit = 1u << 22;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kWaves; ++w) r += red[w];
    return r;   // same value in every thread
}

__device__ void group_barrier(unsigned *ctr, unsigned G, unsigned &gen, unsigned *err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(ctr, 1u);
        const unsigned target = (gen + 1) * G;
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(8);
            if (++spins > kSpinLimit) {
                atomicOr(err, 1u);
                break;
            }
        }
        __threadfence();
    }
    ++gen;
    __syncthreads();
}

template <typename R>
__device__ double tile_energy(const cx<R> *lds, int m, uint64_t base, const BatchTerm *terms,
                              int nt) {
    const int T = 1 << m;
    double acc = 0.0;
    for (int t = 0; t < nt; ++t) {
        const BatchTerm tm = terms[t];
        const int sbase = __popcll(base & tm.z_hi) & 1;
        if (tm.xtop < 0) {
            for (int j = threadIdx.x; j < T; j += kBlock) {
                const cx<R> a = lds[j];
                const double w = double(a.re) * double(a.re) + double(a.im) * double(a.im);
                acc += ((sbase + __popc(uint32_t(j) & tm.zc)) & 1) ? -tm.c * w : tm.c * w;
            }
        } else if (tm.zc == 0 && tm.ph == 0 && sbase == 0) {   // uniform: X factors only
            // both signs +1: the pair gives 2 Re(conj(b) a)
            double v = 0.0;
            for (int g = threadIdx.x; g < (T >> 1); g += kBlock) {
                const uint32_t j = uint32_t(insert_zero(uint64_t(g), tm.xtop));
                const cx<R> pa = lds[j], pb = lds[j ^ tm.xc];
                v += double(pb.re) * double(pa.re) + double(pb.im) * double(pa.im);
            }
            acc += 2.0 * tm.c * v;
        } else {
            for (int g = threadIdx.x; g < (T >> 1); g += kBlock) {
                const uint32_t j = uint32_t(insert_zero(uint64_t(g), tm.xtop));
                const uint32_t jx = j ^ tm.xc;
                const cx<R> pa = lds[j], pb = lds[jx];
                const double ar = pa.re, ai = pa.im, br = pb.re, bi = pb.im;
                const double c1 = br * ar + bi * ai, c2 = br * ai - bi * ar;
                const double sj = ((sbase + __popc(j & tm.zc)) & 1) ? -1.0 : 1.0;
                const double sx = ((sbase + __popc(jx & tm.zc)) & 1) ? -1.0 : 1.0;
                double v;
                switch (tm.ph) {
                case 0: v = (sj + sx) * c1; break;
                case 1: v = -(sj - sx) * c2; break;
                case 2: v = -(sj + sx) * c1; break;
                default: v = (sj - sx) * c2; break;
                }
                acc += tm.c * v;
            }
        }
    }
    return acc;
}

// Run circuit c with `G` cooperating workgroups (this one has rank `rank`).
template <typename R>
__device__ void run_circuit(const BatchArgs &a, int c, int rank, int G, cx<R> *lds, double *red,
                            TileOp *op_slot, unsigned *bar, unsigned &gen) {
    const BatchCircuit C = a.circ[c];
    cx<R> *state = static_cast<cx<R> *>(a.arena) + C.arena_off;
    double acc = 0.0;
    // the phase's tile positions, copied to LDS once per phase: the phase
    // table is in global memory, and vector loads of it inside the tile loop
    // would wait for the stores in flight
    __shared__ uint32_t pos[kTileMaxBits];
    for (int p = C.phase_begin; p < C.phase_begin + C.phase_count; ++p) {
        const BatchPhase &P = a.phases[p];
        if (threadIdx.x < kTileMaxBits) pos[threadIdx.x] = P.pos[threadIdx.x];
        const int m = P.m, flags = P.flags;
        const int op_begin = P.op_begin, op_count = P.op_count;
        const int term_begin = P.term_begin, term_count = P.term_count;
        const uint64_t n_tiles = P.n_tiles;
        __syncthreads();
        const int T = 1 << m;
        const uint64_t off_lo = tile::deposit(uint32_t(threadIdx.x) & uint32_t(T - 1), pos,
                                              m < tile::kLoBits ? m : tile::kLoBits);
        const uint64_t mask = tile::hi_mask(pos, m);
        for (uint64_t t = rank; t < n_tiles; t += G) {
            const uint64_t base = insert_zeros(t, pos, m);
            if (flags & BATCH_INIT) {
                for (int j = threadIdx.x; j < T; j += kBlock) {
                    cx<R> v{R(0), R(0)};
                    if (base == 0 && j == 0) v.re = R(1);
                    lds[j] = v;
                }
            } else {
                tile::tile_load<R>(lds, state, base, off_lo, mask, T);
            }
            __syncthreads();
            tile::apply_ops<R>(lds, m, base, a.ops + op_begin, op_count, op_slot);
            if (term_count) acc += tile_energy<R>(lds, m, base, a.terms + term_begin, term_count);
            if (flags & BATCH_STORE) tile::tile_store<R>(state, lds, base, off_lo, mask, T);
            __syncthreads();
        }
        if (G > 1) group_barrier(bar, G, gen, a.error);
        else __threadfence();
    }
    const double tot = block_sum(acc, red);
    if (G == 1) {
        if (threadIdx.x == 0) a.energy[c] = tot;
    } else {
        if (threadIdx.x == 0) a.partial[size_t(c) * G + rank] = tot;
        group_barrier(bar, G, gen, a.error);
        if (rank == 0 && threadIdx.x == 0) {
            double e = 0.0;
            for (int r = 0; r < G; ++r) e += a.partial[size_t(c) * G + r];
            a.energy[c] = e;
        }
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_batch(const BatchArgs a) {
    extern __shared__ unsigned char smem[];
    __shared__ double red[kWaves];
    __shared__ TileOp op_slot[2];
    cx<R> *lds = reinterpret_cast<cx<R> *>(smem);
    // groups of G workgroups, members on one XCD under round-robin dispatch
    const unsigned G = unsigned(a.G);
    const unsigned xcd = blockIdx.x % 8u, k = blockIdx.x / 8u;
    const unsigned group = xcd + 8u * (k / G);
    const unsigned rank = k % G;
    if (group >= unsigned(a.n_groups)) return;
    unsigned *bar = a.barrier + group;
    unsigned gen = 0;
    for (int jb = a.group_jobs[group]; jb < a.group_jobs[group + 1]; ++jb) {
        const BatchJob &job = a.jobs[jb];
        if (job.kind == 0) {
            const int c = job.circ[rank];
            unsigned g0 = 0;
            if (c >= 0) run_circuit<R>(a, c, 0, 1, lds, red, op_slot, bar, g0);
        } else {
            run_circuit<R>(a, job.circ[0], int(rank), int(G), lds, red, op_slot, bar, gen);
        }
        group_barrier(bar, G, gen, a.error);
    }
}

__global__ void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

int batch_resident_blocks(int dtype, size_t lds_bytes) {
    int nb = 0;
    hipError_t e;
    if (dtype == QC_C64)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<float>, kBlock, lds_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<double>, kBlock, lds_bytes);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_batch(const BatchArgs &a, int dtype, unsigned grid, size_t lds_bytes,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(unsigned((a.n_groups + 1 + 255) / 256)), dim3(256), 0, s,
                       a.barrier, a.n_groups + 1);   // counters + error flag
    const int tok = timer_begin(dtype == QC_C64 ? "batch_c64" : "batch_c128", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_batch<float>), dim3(grid), dim3(kBlock), lds_bytes, s, a);
    else
        hipLaunchKernelGGL((k_batch<double>), dim3(grid), dim3(kBlock), lds_bytes, s, a);
    timer_end(tok, s);
    return hipGetLastError();
}

}  // namespace qcx
