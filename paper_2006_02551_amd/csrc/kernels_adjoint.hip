// Kernels of the loss-gradient path besides the adjoint stage itself (which
// also carries the stage-adjoint update y <- A_{i+1} y + B_i q_hat):
//  - the shell energy 1/2 sum_k J_k sum_q w_q chi (V_q u)^2 (cubature form,
//    eqs. (19)-(20)) and its energy-inner-product gradient P_q (chi V_q u).
// One workgroup per 64-element block, wavefront u = field component u, lane =
// element slot; the operators V_q and P_q^T are staged in LDS and read as
// wave-uniform operands.
#include "device.hpp"

namespace wdg {
namespace {

constexpr int kQmax = 128;

template <int N>
struct OrdA {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
};

template <typename real, int N>
__global__ __launch_bounds__(kThreads) void shell_energy_kernel(ShellParams p) {
    constexpr int Np = OrdA<N>::Np, B = kBlock, EHS = 6 * Np * B;
    __shared__ real sV[kQmax * Np];
    __shared__ double red[kThreads];
    const int Nq = p.Nq, sb = static_cast<int>(blockIdx.x), tid = static_cast<int>(threadIdx.x);
    const int u = tid >> 6, lane = tid & 63;
    for (int i = tid; i < Nq * Np; i += kThreads) sV[i] = static_cast<const real*>(p.Vq)[i];
    __syncthreads();
    const int blk = p.blocks[sb];
    const real* q = static_cast<const real*>(p.q) + static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + lane;
    real uv[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) uv[i] = q[static_cast<size_t>(i) * B];
    const real* chi = static_cast<const real*>(p.chi) + static_cast<size_t>(sb) * Nq * B + lane;
    const double J = p.Jk[static_cast<size_t>(blk) * B + lane];
    double acc = 0.0;
    for (int qq = 0; qq < Nq; ++qq) {
        const real c = chi[static_cast<size_t>(qq) * B];
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

template <typename real, int N>
__global__ __launch_bounds__(kThreads) void shell_inject_kernel(ShellParams p) {
    constexpr int Np = OrdA<N>::Np, B = kBlock, EHS = 6 * Np * B;
    __shared__ real sV[kQmax * Np], sP[kQmax * Np];
    const int Nq = p.Nq, sb = static_cast<int>(blockIdx.x), tid = static_cast<int>(threadIdx.x);
    const int u = tid >> 6, lane = tid & 63;
    for (int i = tid; i < Nq * Np; i += kThreads) {
        sV[i] = static_cast<const real*>(p.Vq)[i];
        sP[i] = static_cast<const real*>(p.PqT)[i];
    }
    __syncthreads();
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
    const real* chi = static_cast<const real*>(p.chi) + static_cast<size_t>(sb) * Nq * B + lane;
    for (int qq = 0; qq < Nq; ++qq) {
        const real c = chi[static_cast<size_t>(qq) * B];
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

template <typename real>
int energy_n(int N, const ShellParams& p, hipStream_t s) {
    const dim3 g(p.nsb), b(kThreads);
    switch (N) {
        case 1: hipLaunchKernelGGL((shell_energy_kernel<real, 1>), g, b, 0, s, p); break;
        case 2: hipLaunchKernelGGL((shell_energy_kernel<real, 2>), g, b, 0, s, p); break;
        case 3: hipLaunchKernelGGL((shell_energy_kernel<real, 3>), g, b, 0, s, p); break;
        case 4: hipLaunchKernelGGL((shell_energy_kernel<real, 4>), g, b, 0, s, p); break;
        default: return static_cast<int>(hipErrorInvalidValue);
    }
    return static_cast<int>(hipGetLastError());
}

template <typename real>
int inject_n(int N, const ShellParams& p, hipStream_t s) {
    const dim3 g(p.nsb), b(kThreads);
    switch (N) {
        case 1: hipLaunchKernelGGL((shell_inject_kernel<real, 1>), g, b, 0, s, p); break;
        case 2: hipLaunchKernelGGL((shell_inject_kernel<real, 2>), g, b, 0, s, p); break;
        case 3: hipLaunchKernelGGL((shell_inject_kernel<real, 3>), g, b, 0, s, p); break;
        case 4: hipLaunchKernelGGL((shell_inject_kernel<real, 4>), g, b, 0, s, p); break;
        default: return static_cast<int>(hipErrorInvalidValue);
    }
    return static_cast<int>(hipGetLastError());
}

}  // namespace

int launch_shell_energy(int precision, int N, const ShellParams& p, hipStream_t s) {
    if (p.Nq > kQmax) return static_cast<int>(hipErrorInvalidValue);
    if (p.nsb == 0) return 0;
    return precision == 0 ? energy_n<double>(N, p, s) : energy_n<float>(N, p, s);
}

int launch_sum_into(const double* partial, int n, double scale, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(256), 0, s, partial, n, scale, acc);
    return static_cast<int>(hipGetLastError());
}

int launch_shell_inject(int precision, int N, const ShellParams& p, hipStream_t s) {
    if (p.Nq > kQmax) return static_cast<int>(hipErrorInvalidValue);
    if (p.nsb == 0) return 0;
    return precision == 0 ? inject_n<double>(N, p, s) : inject_n<float>(N, p, s);
}

}  // namespace wdg
