// Kernels of the loss-gradient path besides the adjoint stage itself (which
// also carries the stage-adjoint update y <- A_{i+1} y + B_i q_hat):
//  - the shell energy 1/2 sum_k J_k sum_q w_q chi (V_q u)^2 (cubature form,
//    eqs. (19)-(20)) and its energy-inner-product gradient P_q (chi V_q u).
// One workgroup per 64-element block, wavefront u = field component u, lane =
// element slot; the operators V_q and P_q^T and the block's shell indicator
// are staged in LDS (operators read as wave-uniform operands).
#include "device.hpp"

namespace wdg {
namespace {

constexpr int kQmax = 128;

template <int N>
struct OrdA {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
};

// Dynamic LDS of the shell kernels: V_q (and P_q^T) [Nq][Np], then, when CL, the block's shell indicator
// [Nq][B] (staged with the operators, so the cubature loop waits for no global load).
template <typename real>
constexpr size_t shell_lds(int Nq, int Np, int nops, bool cl) {
    return (static_cast<size_t>(nops) * Nq * Np + (cl ? static_cast<size_t>(Nq) * kBlock : 0)) * sizeof(real);
}
constexpr size_t kShellLdsMax = 64 * 1024;

template <typename real, int N, bool CL>
__global__ __launch_bounds__(kThreads) void shell_energy_kernel(ShellParams p) {
    constexpr int Np = OrdA<N>::Np, B = kBlock, EHS = 6 * Np * B;
    extern __shared__ __attribute__((aligned(16))) char dyn[];
    real* sV = reinterpret_cast<real*>(dyn);
    real* sC = sV + p.Nq * Np;
    __shared__ double red[kThreads];
    const int Nq = p.Nq, sb = static_cast<int>(blockIdx.x), tid = static_cast<int>(threadIdx.x);
    const int u = tid >> 6, lane = tid & 63;
    const real* chig = static_cast<const real*>(p.chi) + static_cast<size_t>(sb) * Nq * B;
    for (int i = tid; i < Nq * Np; i += kThreads) sV[i] = static_cast<const real*>(p.Vq)[i];
    if (CL)
        for (int i = tid; i < Nq * B; i += kThreads) sC[i] = chig[i];
    const int blk = p.blocks[sb];
    const real* q = static_cast<const real*>(p.q) + static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + lane;
    real uv[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) uv[i] = q[static_cast<size_t>(i) * B];
    const double J = p.Jk[static_cast<size_t>(blk) * B + lane];
    __syncthreads();
    const real* chi;
    if constexpr (CL) chi = sC + lane;
    else chi = chig + lane;
    double acc = 0.0;
    for (int qq = 0; qq < Nq; ++qq) {
        const real c = chi[qq * B];
        real v = real(0);
#pragma unroll
        for (int jj = 0; jj < Np; ++jj) v += sV[qq * Np + jj] * uv[jj];
        acc += static_cast<double>(c) * p.cub_w[qq] * static_cast<double>(v) * static_cast<double>(v);
    }
    red[tid] = J * acc;
    __syncthreads();
    // fixed-order tree over the 384 values: 384 -> 256, then halving
    for (int w = 256; w >= 1; w >>= 1) {
        if (tid < w && tid + w < kThreads) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) p.partial[sb] = red[0];
}

__global__ __launch_bounds__(256) void sum_into_kernel(const double* partial, int n, double scale, double* acc) {
    __shared__ double red[256];
    const int tid = static_cast<int>(threadIdx.x);
    double s = 0.0;
    for (int i = tid; i < n; i += 256) s += partial[i];
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) *acc += scale * red[0];
}

template <typename real, int N, bool CL>
__global__ __launch_bounds__(kThreads) void shell_inject_kernel(ShellParams p) {
    constexpr int Np = OrdA<N>::Np, B = kBlock, EHS = 6 * Np * B;
    extern __shared__ __attribute__((aligned(16))) char dyn[];
    real* sV = reinterpret_cast<real*>(dyn);
    real* sP = sV + p.Nq * Np;
    real* sC = sP + p.Nq * Np;
    const int Nq = p.Nq, sb = static_cast<int>(blockIdx.x), tid = static_cast<int>(threadIdx.x);
    const int u = tid >> 6, lane = tid & 63;
    const real* chig = static_cast<const real*>(p.chi) + static_cast<size_t>(sb) * Nq * B;
    for (int i = tid; i < Nq * Np; i += kThreads) {
        sV[i] = static_cast<const real*>(p.Vq)[i];
        sP[i] = static_cast<const real*>(p.PqT)[i];
    }
    if (CL)
        for (int i = tid; i < Nq * B; i += kThreads) sC[i] = chig[i];
    const int blk = p.blocks[sb];
    const size_t off = static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + lane;
    const real* q = static_cast<const real*>(p.q) + off;
    real* qh = static_cast<real*>(p.q_hat) + off;
    real uv[Np], gv[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) {
        uv[i] = q[static_cast<size_t>(i) * B];
        gv[i] = real(0);
    }
    __syncthreads();
    const real* chi;
    if constexpr (CL) chi = sC + lane;
    else chi = chig + lane;
    for (int qq = 0; qq < Nq; ++qq) {
        const real c = chi[qq * B];
        real v = real(0);
#pragma unroll
        for (int jj = 0; jj < Np; ++jj) v += sV[qq * Np + jj] * uv[jj];
        v *= c;
#pragma unroll
        for (int i = 0; i < Np; ++i) gv[i] += sP[qq * Np + i] * v;
    }
    const real dt = static_cast<real>(p.dt);
#pragma unroll
    for (int i = 0; i < Np; ++i) qh[static_cast<size_t>(i) * B] += dt * gv[i];
}

template <typename real, int N>
int shell_launch(bool inject, const ShellParams& p, hipStream_t s) {
    constexpr int Np = OrdA<N>::Np;
    const int nops = inject ? 2 : 1;
    const dim3 g(p.nsb), b(kThreads);
    // the indicator goes to LDS with the operators wherever both fit in the default 64 KiB
    const bool cl = shell_lds<real>(p.Nq, Np, nops, true) <= kShellLdsMax;
    const size_t lds = shell_lds<real>(p.Nq, Np, nops, cl);
    if (lds > kShellLdsMax) return static_cast<int>(hipErrorInvalidValue);
    if (inject) {
        if (cl) hipLaunchKernelGGL((shell_inject_kernel<real, N, true>), g, b, lds, s, p);
        else hipLaunchKernelGGL((shell_inject_kernel<real, N, false>), g, b, lds, s, p);
    } else {
        if (cl) hipLaunchKernelGGL((shell_energy_kernel<real, N, true>), g, b, lds, s, p);
        else hipLaunchKernelGGL((shell_energy_kernel<real, N, false>), g, b, lds, s, p);
    }
    return static_cast<int>(hipGetLastError());
}

template <typename real>
int shell_n(int N, bool inject, const ShellParams& p, hipStream_t s) {
    switch (N) {
        case 1: return shell_launch<real, 1>(inject, p, s);
        case 2: return shell_launch<real, 2>(inject, p, s);
        case 3: return shell_launch<real, 3>(inject, p, s);
        case 4: return shell_launch<real, 4>(inject, p, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

}  // namespace

int launch_shell_energy(int precision, int N, const ShellParams& p, hipStream_t s) {
    if (p.Nq > kQmax) return static_cast<int>(hipErrorInvalidValue);
    if (p.nsb == 0) return 0;
    return precision == 0 ? shell_n<double>(N, false, p, s) : shell_n<float>(N, false, p, s);
}

int launch_sum_into(const double* partial, int n, double scale, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(256), 0, s, partial, n, scale, acc);
    return static_cast<int>(hipGetLastError());
}

int launch_shell_inject(int precision, int N, const ShellParams& p, hipStream_t s) {
    if (p.Nq > kQmax) return static_cast<int>(hipErrorInvalidValue);
    if (p.nsb == 0) return 0;
    return precision == 0 ? shell_n<double>(N, true, p, s) : shell_n<float>(N, true, p, s);
}

}  // namespace wdg
