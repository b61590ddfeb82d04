// Adjoint-method gradient kernels (Jones & Gacon, arXiv:2009.02823; the
// QCLAB paper itself has no gradients).
//
// For E(theta) = <phi|H|phi>, phi = U_L ... U_1 psi and a parametrised gate
// U_k = exp(-i theta G / 2) with G in {X, Y, Z}:
//   dE/dtheta_k = 2 Re <lam_k| dU_k/dtheta |phi_{k-1}> = Im <lam_k| G |phi_k>,
// where phi_k is the state after gate k and lam_k = U_{k+1}^+ .. U_L^+ H phi.
// The backward sweep keeps (phi, lam) at step k, takes the FP64 reduction
// Im <lam|G|phi> and un-applies U_k to both vectors in the same pass over
// memory (read 2 vectors, write 2 vectors).
#include "qc_internal.h"

#include "../../include/qc.h"

namespace qcx {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// lam = H psi = sum_t c_t i^ny (-1)^popc((j^x) & z) psi_{j^x}
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pauli_apply(const cx<R> *psi, cx<R> *out,
                                                        uint64_t count,
                                                        const PauliTermDev *terms, int nt) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < count; j += stride) {
        const cx<R> pj = psi[j];
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < nt; ++t) {
            const PauliTermDev T = terms[t];
            const uint64_t k = j ^ T.x;
            const cx<R> a = T.x ? psi[k] : pj;
            const double s = (__popcll(k & T.z) & 1) ? -T.c : T.c;
            double vr = s * double(a.re), vi = s * double(a.im);
            switch (T.ph) {
            case 0: break;
            case 1: { const double tr = -vi; vi = vr; vr = tr; } break;
            case 2: vr = -vr; vi = -vi; break;
            default: { const double tr = vi; vi = -vr; vr = tr; } break;
            }
            ar += vr;
            ai += vi;
        }
        out[j] = cx<R>{R(ar), R(ai)};
    }
}

// One backward step for a one-qubit parametrised gate on bit p with
// generator G (1 = X, 2 = Y, 3 = Z): partial Im <lam|G|phi> per block, then
// phi <- Ud phi, lam <- Ud lam with Ud = U^+.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adjoint_step(cx<R> *phi, cx<R> *lam, uint64_t n_pairs,
                                                         int p, int gen, const Mat2d ud,
                                                         double *partial) {
    __shared__ double lds[kWaves];
    double acc = 0.0;
    const uint64_t bit = uint64_t(1) << p;
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < n_pairs; g += stride) {
        const uint64_t i0 = insert_zero(g, p), i1 = i0 | bit;
        const cx<R> f0 = phi[i0], f1 = phi[i1], l0 = lam[i0], l1 = lam[i1];
        const double f0r = f0.re, f0i = f0.im, f1r = f1.re, f1i = f1.im;
        const double l0r = l0.re, l0i = l0.im, l1r = l1.re, l1i = l1.im;
        // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
        if (gen == 3) {
            acc += (l0r * f0i - l0i * f0r) - (l1r * f1i - l1i * f1r);
        } else if (gen == 1) {
            acc += (l0r * f1i - l0i * f1r) + (l1r * f0i - l1i * f0r);
        } else {
            acc += -(l0r * f1r + l0i * f1i) + (l1r * f0r + l1i * f0i);
        }
        const R u0r = R(ud.re[0]), u0i = R(ud.im[0]), u1r = R(ud.re[1]), u1i = R(ud.im[1]);
        const R u2r = R(ud.re[2]), u2i = R(ud.im[2]), u3r = R(ud.re[3]), u3i = R(ud.im[3]);
        const cx<R> U0{u0r, u0i}, U1{u1r, u1i}, U2{u2r, u2i}, U3{u3r, u3i};
        const cx<R> zero{R(0), R(0)};
        phi[i0] = cfma(U1, f1, cfma(U0, f0, zero));
        phi[i1] = cfma(U3, f1, cfma(U2, f0, zero));
        lam[i0] = cfma(U1, l1, cfma(U0, l0, zero));
        lam[i1] = cfma(U3, l1, cfma(U2, l0, zero));
    }
    double v = wave_sum(acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kWaves; ++w) r += lds[w];
        partial[blockIdx.x] = r;
    }
}

// g_op[i] = sum of row i of the partials (fixed order), then
// grad[p] = sum over the ops of parameter p (CSR, op order).
__global__ __launch_bounds__(kBlock) void k_grad_rows(const double *partial, int cols,
                                                      double *g_op) {
    __shared__ double lds[kWaves];
    const int row = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < cols; c += kBlock) acc += partial[size_t(row) * cols + c];
    double v = wave_sum(acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < kWaves; ++w) r += lds[w];
        g_op[row] = r;
    }
}

__global__ void k_grad_scatter(const double *g_op, const int *ptr, const int *idx, int n_params,
                               double *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_params) return;
    double s = 0.0;
    for (int k = ptr[p]; k < ptr[p + 1]; ++k) s += g_op[idx[k]];
    grad[p] = s;
}

unsigned grid_for(uint64_t items) {
    uint64_t b = (items + kBlock * 8 - 1) / (kBlock * 8);
    if (b < 1) b = 1;
    if (b > unsigned(kReduceBlocks)) b = kReduceBlocks;
    return unsigned(b);
}

}  // namespace

unsigned adjoint_grid(int n) { return grid_for(uint64_t(1) << (n - 1)); }

hipError_t launch_pauli_apply(const void *psi, void *out, int dtype, int n,
                              const PauliTermDev *terms, int nt, hipStream_t s) {
    const uint64_t count = uint64_t(1) << n;
    uint64_t g = (count + kBlock * 4 - 1) / (kBlock * 4);
    if (g > 256u * 64u) g = 256u * 64u;
    const int tok = timer_begin("pauli_apply", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_pauli_apply<float>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                           static_cast<const cx<float> *>(psi), static_cast<cx<float> *>(out), count,
                           terms, nt);
    else
        hipLaunchKernelGGL((k_pauli_apply<double>), dim3(unsigned(g)), dim3(kBlock), 0, s,
                           static_cast<const cx<double> *>(psi), static_cast<cx<double> *>(out),
                           count, terms, nt);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(void *phi, void *lam, int dtype, int n, int p, int gen,
                               const Mat2d &ud, double *partial, hipStream_t s) {
    const uint64_t pairs = uint64_t(1) << (n - 1);
    const unsigned grid = grid_for(pairs);
    const int tok = timer_begin("adjoint_step", s);
    if (dtype == QC_C64)
        hipLaunchKernelGGL((k_adjoint_step<float>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<float> *>(phi), static_cast<cx<float> *>(lam), pairs, p, gen,
                           ud, partial);
    else
        hipLaunchKernelGGL((k_adjoint_step<double>), dim3(grid), dim3(kBlock), 0, s,
                           static_cast<cx<double> *>(phi), static_cast<cx<double> *>(lam), pairs, p,
                           gen, ud, partial);
    timer_end(tok, s);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(const double *partial, int rows, int cols, double *g_op,
                                const int *ptr, const int *idx, int n_params, double *grad,
                                hipStream_t s) {
    if (rows > 0)
        hipLaunchKernelGGL(k_grad_rows, dim3(unsigned(rows)), dim3(kBlock), 0, s, partial, cols,
                           g_op);
    if (n_params > 0)
        hipLaunchKernelGGL(k_grad_scatter, dim3(unsigned((n_params + 255) / 256)), dim3(256), 0,
                           s, g_op, ptr, idx, n_params, grad);
    return hipGetLastError();
}

}  // namespace qcx
