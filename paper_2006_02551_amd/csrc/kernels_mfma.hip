// Matrix-core (MFMA) form of the fused stage kernel for gfx950.
//
// Same mathematics and memory layout as the scalar-operand kernel in
// kernels.hip (eqs. (26)-(29) with the upwind curl of eqs. (15)-(17), the
// weight-adjusted inverse mass of eq. (21) and the LSERK4 update), but every
// small dense product runs on V_MFMA_F64_16X16X4_F64 / V_MFMA_F32_16X16X4_F32:
//
//   Out (M x 16 elements) = Op (M x K) * X (K x 16 elements)
//
// A wavefront owns a tile of 16 elements (the columns).  The reference
// operators are the A operands; they are stored on the host in fragment
// order (tile p, k-step s, lane), copied once per workgroup into LDS and read
// with one 64-lane LDS load per fragment, reused across the six field
// components.  Field data are the B operands.
//
// Register chaining.  Lane l = 16 g + j holds column j; an MFMA result keeps
// four values per lane (register v).  The host permutes the rows of every
// operator so that register v of M-tile p in lane group g holds quantity
//   n(p, g, v) = 16 p + 4 v + g
// (node or cubature point), which is exactly the B operand of k-step 4 p + v
// in natural order.  Results therefore feed the next product with no data
// movement: V_q -> pointwise PML coefficients -> P_q -> V_q -> P_q, and the
// right-hand side accumulates LIFT, curl and P_q terms in one set of
// registers.  The rows held by register v are g + 4 v for the FP64 MFMA and
// 4 g + v for the FP32 MFMA; the host applies the matching permutation.
//
// Per PML tile and component u (f = E or H, P its auxiliary field):
//   A. VF = V_q f_u, VP = V_q P_u; t1 = b VF + c VP, t2 = kappa^-1 VF - d VP
//      (eq. (9) at the cubature points); rhs_P = P_q t2 (then its LSERK
//      update); R_u = -P_q t1
//   B. R += LIFT (Fscale * upwind flux); the flux is computed directly in
//      B-operand layout, one face node per lane group and k-step
//   C. R_u += D_r G_r + D_s G_s + D_t G_t, G_d = metric-weighted components
//   D. rhs_u = P_q a^-1 V_q R_u (PML tiles), then the LSERK update.
#include "device.hpp"

namespace wdg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename real>
struct Mma;
template <>
struct Mma<double> {
    using v4 = v4d;
    static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mma<float> {
    using v4 = v4f;
    static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <int N>
struct Ord {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

__device__ __forceinline__ int remap_block(int bid, int nblk_pml, int nblk) {
    int base = 0, n = nblk_pml;
    if (bid >= nblk_pml) {
        base = nblk_pml;
        n = nblk - nblk_pml;
    }
    const int j = bid - base;
    const int x = j & 7, i = j >> 3;
    const int q = n >> 3, r = n & 7;
    return base + x * q + (x < r ? x : r) + i;
}

template <typename real, int N, int QT, bool KAPPA>
__global__ __launch_bounds__(kMfmaThreads) void stage_mfma_kernel(StageParams p) {
    using M = Mma<real>;
    using v4 = typename M::v4;
    constexpr int Np = Ord<N>::Np, Nfp = Ord<N>::Nfp, B = kBlock;
    constexpr int PT = (Np + 15) / 16;  // node tiles
    constexpr int SP = (Np + 3) / 4;    // k-steps over nodes
    constexpr int SQM = 4 * QT;         // k-steps reserved over cubature points
    constexpr int SF = Nfp;             // k-steps over the 4 Nfp face nodes
    constexpr int OFF_VQ = 0;
    constexpr int OFF_PQ = OFF_VQ + QT * SP;
    constexpr int OFF_D = OFF_PQ + PT * SQM;
    constexpr int OFF_L = OFF_D + 3 * PT * SP;
    constexpr int NFRAG = OFF_L + PT * SF;
    constexpr int EHS = 6 * Np * B;
    __shared__ real fr[NFRAG * 64];

    // operators to LDS (fragment order is prepared on the host)
    {
        const real* __restrict__ src = static_cast<const real*>(p.frags);
        for (int i = static_cast<int>(threadIdx.x); i < NFRAG * 64; i += kMfmaThreads) fr[i] = src[i];
    }
    __syncthreads();

    const int lane = static_cast<int>(threadIdx.x) & 63;
    const int wave = static_cast<int>(threadIdx.x) >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int blk = __builtin_amdgcn_readfirstlane(remap_block(blockIdx.x, p.nblk_pml, p.nblk));
    const bool pml = blk < p.nblk_pml;
    const int e = 16 * wave + j;  // element slot inside the block
    const int Nq = p.Nq;
    const int SQ = (Nq + 3) / 4;

    const real* __restrict__ qin = static_cast<const real*>(p.q_in);
    const real* __restrict__ qe = qin + static_cast<size_t>(blk) * EHS + e;
    const real* __restrict__ geo = static_cast<const real*>(p.geo) + static_cast<size_t>(blk) * kGeo * B + e;
    const size_t pbase = static_cast<size_t>(p.nblk) * EHS + static_cast<size_t>(blk) * EHS + e;
    real* __restrict__ rs = static_cast<real*>(p.res);
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    const real rkA = static_cast<real>(p.rk_a), rkB = static_cast<real>(p.rk_b), dt = static_cast<real>(p.dt);
    const bool read_res = p.read_res != 0;

    auto frag = [&](int f) -> real { return fr[f * 64 + lane]; };

    v4 R[6][PT];
#pragma unroll
    for (int u = 0; u < 6; ++u)
#pragma unroll
        for (int t = 0; t < PT; ++t) R[u][t] = v4{0, 0, 0, 0};

    // ---------------- A. PML terms at the cubature points
    if (pml) {
        const real* __restrict__ sg = static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + e;
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e : nullptr;
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int ax = (u < 3) ? u : u - 3;
            const int bb = (ax == 2) ? 0 : ax + 1;
            const int cc = (ax == 0) ? 2 : ax - 1;
            real bf[SP], bp[SP];
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                const int node = 4 * s + g;
                const bool ok = (SP * 4 == Np) || node < Np;
                bf[s] = ok ? qe[(u * Np + node) * B] : real(0);
                bp[s] = ok ? qin[pbase + static_cast<size_t>(u * Np + node) * B] : real(0);
            }
            v4 VF[QT], VP[QT];
#pragma unroll
            for (int t = 0; t < QT; ++t) VF[t] = VP[t] = v4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < SP; ++s)
#pragma unroll
                for (int t = 0; t < QT; ++t) {
                    const real a = frag(OFF_VQ + t * SP + s);
                    VF[t] = M::run(a, bf[s], VF[t]);
                    VP[t] = M::run(a, bp[s], VP[t]);
                }
            // eq. (9) at cubature point q = 16 t + 4 v + g: VF <- -t1, VP <- t2
#pragma unroll
            for (int t = 0; t < QT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 16 * t + 4 * v + g;
                    real t1 = real(0), t2 = real(0);
                    if (q < Nq) {
                        const real sa = sg[(ax * Nq + q) * B], sb = sg[(bb * Nq + q) * B], sc = sg[(cc * Nq + q) * B];
                        real bq, cq, dq, kinv;
                        if (KAPPA) {
                            const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                            kinv = real(1) / ka;
                            const real aa = kb * kc * kinv;
                            bq = (sb * kc + sc * kb - aa * sa) * kinv;
                            cq = sb * sc - bq * sa;
                            dq = sa * kinv;
                        } else {
                            kinv = real(1);
                            bq = sb + sc - sa;
                            cq = sb * sc - bq * sa;
                            dq = sa;
                        }
                        const real vf = VF[t][v], vp = VP[t][v];
                        t1 = bq * vf + cq * vp;
                        t2 = kinv * vf - dq * vp;
                    }
                    VF[t][v] = -t1;
                    VP[t][v] = t2;
                }
            // rhs_P = P_q t2 and R_u = -P_q t1
            v4 RP[PT];
#pragma unroll
            for (int t = 0; t < PT; ++t) RP[t] = v4{0, 0, 0, 0};
#pragma unroll
            for (int tq = 0; tq < QT; ++tq)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int sq = 4 * tq + v;
                    if (sq < SQ) {
#pragma unroll
                        for (int t = 0; t < PT; ++t) {
                            const real a = frag(OFF_PQ + t * SQM + sq);
                            RP[t] = M::run(a, VP[tq][v], RP[t]);
                            R[u][t] = M::run(a, VF[tq][v], R[u][t]);
                        }
                    }
                }
            // LSERK update of the auxiliary component u
#pragma unroll
            for (int t = 0; t < PT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int node = 16 * t + 4 * v + g;
                    if (node < Np) {
                        const size_t idx = pbase + static_cast<size_t>(u * Np + node) * B;
                        real r = dt * RP[t][v];
                        if (read_res) r += rkA * rs[idx];
                        rs[idx] = r;
                        qo[idx] = qin[idx] + rkB * r;
                    }
                }
        }
    }

    // ---------------- B. upwind flux lifted to the volume
    {
        const int* __restrict__ nbr = p.nbr + static_cast<size_t>(blk) * 4 * Nfp * B + e;
        const real alpha = static_cast<real>(p.alpha);
#pragma unroll 2
        for (int s = 0; s < SF; ++s) {
            const int fn = 4 * s + g;  // face node (face fc, index m)
            const int fc = fn / Nfp;
            const int jn = p.fmask[fn];
            const real Ex = qe[(0 * Np + jn) * B], Ey = qe[(1 * Np + jn) * B], Ez = qe[(2 * Np + jn) * B];
            const real Hx = qe[(3 * Np + jn) * B], Hy = qe[(4 * Np + jn) * B], Hz = qe[(5 * Np + jn) * B];
            const int vv = nbr[fn * B];
            const int off = vv >= 0 ? vv : ~vv;
            const real sE = vv >= 0 ? real(1) : real(-1);
            const real* __restrict__ qp = qin + off;
            const real dEx = Ex - sE * qp[0 * Np * B], dEy = Ey - sE * qp[1 * Np * B], dEz = Ez - sE * qp[2 * Np * B];
            const real dHx = Hx - qp[3 * Np * B], dHy = Hy - qp[4 * Np * B], dHz = Hz - qp[5 * Np * B];
            const real nx = geo[(9 + 4 * fc) * B], ny = geo[(10 + 4 * fc) * B], nz = geo[(11 + 4 * fc) * B];
            const real hs = real(0.5) * geo[(12 + 4 * fc) * B];
            const real ndE = nx * dEx + ny * dEy + nz * dEz;
            const real ndH = nx * dHx + ny * dHy + nz * dHz;
            real fl[6];
            fl[0] = hs * (-(ny * dHz - nz * dHy) + alpha * (nx * ndE - dEx));
            fl[1] = hs * (-(nz * dHx - nx * dHz) + alpha * (ny * ndE - dEy));
            fl[2] = hs * (-(nx * dHy - ny * dHx) + alpha * (nz * ndE - dEz));
            fl[3] = hs * ((ny * dEz - nz * dEy) + alpha * (nx * ndH - dHx));
            fl[4] = hs * ((nz * dEx - nx * dEz) + alpha * (ny * ndH - dHy));
            fl[5] = hs * ((nx * dEy - ny * dEx) + alpha * (nz * ndH - dHz));
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                const real a = frag(OFF_L + t * SF + s);
#pragma unroll
                for (int c = 0; c < 6; ++c) R[c][t] = M::run(a, fl[c], R[c][t]);
            }
        }
    }

    // ---------------- C. volume curl: +curl H (E components), -curl E (H components)
    {
        real mt[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) mt[d] = geo[d * B];
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int ax = (u < 3) ? u : u - 3;
            const int bb = (ax == 2) ? 0 : ax + 1;
            const int cc = (ax == 0) ? 2 : ax - 1;
            const int fo = (u < 3) ? 3 : 0;
            const real sgn = (u < 3) ? real(1) : real(-1);
            const real rb = sgn * mt[bb], rc = sgn * mt[cc];
            const real sb = sgn * mt[3 + bb], sc = sgn * mt[3 + cc];
            const real tb = sgn * mt[6 + bb], tc = sgn * mt[6 + cc];
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                const int node = 4 * s + g;
                const bool ok = (SP * 4 == Np) || node < Np;
                const real xb = ok ? qe[((fo + bb) * Np + node) * B] : real(0);
                const real xc = ok ? qe[((fo + cc) * Np + node) * B] : real(0);
                const real gr = rb * xc - rc * xb, gs = sb * xc - sc * xb, gt = tb * xc - tc * xb;
#pragma unroll
                for (int t = 0; t < PT; ++t) {
                    R[u][t] = M::run(frag(OFF_D + (0 * PT + t) * SP + s), gr, R[u][t]);
                    R[u][t] = M::run(frag(OFF_D + (1 * PT + t) * SP + s), gs, R[u][t]);
                    R[u][t] = M::run(frag(OFF_D + (2 * PT + t) * SP + s), gt, R[u][t]);
                }
            }
        }
    }

    // ---------------- dipole source on the electric components
    {
        const int slot = p.src_slot[blk];
        if (slot >= 0) {
            const real gsrc = static_cast<real>(p.src_g);
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const real* __restrict__ S = static_cast<const real*>(p.src) + (static_cast<size_t>(slot) * 3 + u) * Np * B + e;
#pragma unroll
                for (int t = 0; t < PT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int node = 16 * t + 4 * v + g;
                        if (node < Np) R[u][t][v] -= gsrc * S[node * B];
                    }
            }
        }
    }

    // ---------------- D. weight-adjusted inverse mass on PML tiles: rhs_u = P_q a^-1 V_q R_u
    if (pml) {
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e : nullptr;
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            v4 Z[QT];
#pragma unroll
            for (int t = 0; t < QT; ++t) Z[t] = v4{0, 0, 0, 0};
#pragma unroll
            for (int tp = 0; tp < PT; ++tp)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int sp = 4 * tp + v;
                    if (sp < SP) {
#pragma unroll
                        for (int t = 0; t < QT; ++t) Z[t] = M::run(frag(OFF_VQ + t * SP + sp), R[u][tp][v], Z[t]);
                    }
                }
            if (KAPPA) {
                const int ax = (u < 3) ? u : u - 3;
                const int bb = (ax == 2) ? 0 : ax + 1;
                const int cc = (ax == 0) ? 2 : ax - 1;
#pragma unroll
                for (int t = 0; t < QT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int q = 16 * t + 4 * v + g;
                        if (q < Nq) {
                            const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                            Z[t][v] *= ka / (kb * kc);
                        }
                    }
            }
            v4 O[PT];
#pragma unroll
            for (int t = 0; t < PT; ++t) O[t] = v4{0, 0, 0, 0};
#pragma unroll
            for (int tq = 0; tq < QT; ++tq)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int sq = 4 * tq + v;
                    if (sq < SQ) {
#pragma unroll
                        for (int t = 0; t < PT; ++t) O[t] = M::run(frag(OFF_PQ + t * SQM + sq), Z[tq][v], O[t]);
                    }
                }
#pragma unroll
            for (int t = 0; t < PT; ++t) R[u][t] = O[t];
        }
    }

    // ---------------- LSERK4 update of E and H
    {
        const size_t eb = static_cast<size_t>(blk) * EHS + e;
#pragma unroll
        for (int u = 0; u < 6; ++u)
#pragma unroll
            for (int t = 0; t < PT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int node = 16 * t + 4 * v + g;
                    if (node < Np) {
                        const size_t idx = eb + static_cast<size_t>(u * Np + node) * B;
                        real r = dt * R[u][t][v];
                        if (read_res) r += rkA * rs[idx];
                        rs[idx] = r;
                        qo[idx] = qin[idx] + rkB * r;
                    }
                }
    }
}

template <typename real, int N, int QT, bool K>
int launch_t(const StageParams& p, hipStream_t s) {
    hipLaunchKernelGGL((stage_mfma_kernel<real, N, QT, K>), dim3(p.nblk), dim3(kMfmaThreads), 0, s, p);
    return static_cast<int>(hipGetLastError());
}

template <typename real, int N, int QT>
int launch_k(bool k, const StageParams& p, hipStream_t s) {
    return k ? launch_t<real, N, QT, true>(p, s) : launch_t<real, N, QT, false>(p, s);
}

template <typename real>
int launch_r(int N, int QT, bool k, const StageParams& p, hipStream_t s) {
    switch (N * 10 + QT) {
        case 11: return launch_k<real, 1, 1>(k, p, s);
        case 12: return launch_k<real, 1, 2>(k, p, s);
        case 21: return launch_k<real, 2, 1>(k, p, s);
        case 22: return launch_k<real, 2, 2>(k, p, s);
        case 32: return launch_k<real, 3, 2>(k, p, s);
        case 33: return launch_k<real, 3, 3>(k, p, s);
        case 43: return launch_k<real, 4, 3>(k, p, s);
        case 44: return launch_k<real, 4, 4>(k, p, s);
        default: return -1;
    }
}

}  // namespace

bool mfma_supported(int N, int Nq) {
    const int QT = (Nq + 15) / 16;
    switch (N * 10 + QT) {
        case 11: case 12: case 21: case 22: case 32: case 33: case 43: case 44: return true;
        default: return false;
    }
}

int launch_stage_mfma(int precision, int N, bool has_kappa, const StageParams& p, hipStream_t s) {
    const int QT = (p.Nq + 15) / 16;
    return precision == 0 ? launch_r<double>(N, QT, has_kappa, p, s) : launch_r<float>(N, QT, has_kappa, p, s);
}

}  // namespace wdg
