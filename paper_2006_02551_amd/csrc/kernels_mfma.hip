// Matrix-core (MFMA) form of the fused stage kernel for gfx950.
//
// Same mathematics and memory layout as the scalar-operand kernel in
// kernels.hip (eqs. (26)-(29) with the upwind curl of eqs. (15)-(17), the
// weight-adjusted inverse mass of eq. (21) and the LSERK4 update), but every
// small dense product runs on V_MFMA_F64_16X16X4_F64 / V_MFMA_F32_16X16X4_F32:
//
//   Out (M x 16 elements) = Op (M x K) * X (K x 16 elements)
//
// A workgroup owns a tile of 16 elements (the columns) and has six
// wavefronts, one per field component u.  The reference operators are the A
// operands; they are stored on the host in fragment order (tile p, k-step s,
// lane), copied once per workgroup into LDS and read with one 64-lane LDS load
// per fragment.  Field data are the B operands.  The upwind flux of all six
// components is computed once per tile by the whole workgroup (one face node
// and element per thread) and shared through LDS.
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
// Per PML tile, wavefront u (f = E or H, P its auxiliary field):
//   B. R = LIFT (Fscale * upwind flux), flux read from LDS in B layout
//   C. R += D_r G_r + D_s G_s + D_t G_t, G_d = metric-weighted components
//   A. VF = V_q f_u, VP = V_q P_u; t1 = b VF + c VP, t2 = kappa^-1 VF - d VP
//      (eq. (9) at the cubature points); rhs_P = P_q t2 (then its LSERK
//      update); R -= P_q t1
//   D. rhs_u = P_q a^-1 V_q R (PML tiles), then the LSERK update.
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

// Tiles: every element block of 64 slots is four tiles of 16; PML tiles first.
__device__ __forceinline__ int remap_tile(int bid, int ntile_pml, int ntile) {
    int base = 0, n = ntile_pml;
    if (bid >= ntile_pml) {
        base = ntile_pml;
        n = ntile - ntile_pml;
    }
    const int jj = bid - base;
    const int x = jj & 7, i = jj >> 3;
    const int q = n >> 3, r = n & 7;
    return base + x * q + (x < r ? x : r) + i;
}

template <typename real, int N, int QT, bool KAPPA>
__global__ __launch_bounds__(kMfmaThreads) void stage_mfma_kernel(StageParams p) {
    using M = Mma<real>;
    using v4 = typename M::v4;
    constexpr int Np = Ord<N>::Np, Nfp = Ord<N>::Nfp, B = kBlock;
    constexpr int NF = 4 * Nfp;         // face nodes per element
    constexpr int PT = (Np + 15) / 16;  // node tiles
    constexpr int SP = (Np + 3) / 4;    // k-steps over nodes
    constexpr int SQM = 4 * QT;         // k-steps reserved over cubature points
    constexpr int SF = Nfp;             // k-steps over the face nodes
    constexpr int OFF_VQ = 0;
    constexpr int OFF_PQ = OFF_VQ + QT * SP;
    constexpr int OFF_D = OFF_PQ + PT * SQM;
    constexpr int OFF_L = OFF_D + 3 * PT * SP;
    constexpr int NFRAG = OFF_L + PT * SF;
    constexpr int EHS = 6 * Np * B;
    constexpr int FIT = (NF * 16 + kMfmaThreads - 1) / kMfmaThreads;  // flux items per thread
    constexpr int NCHUNK = frag_chunks(NFRAG, sizeof(real));          // 1 KiB chunks of fragments
    __shared__ __attribute__((aligned(16))) real fr[NCHUNK * 1024 / sizeof(real)];
    __shared__ real fl[6 * NF * 16];  // flux [component][face node][element of the tile]

    const int tid = static_cast<int>(threadIdx.x);
    const int tile = __builtin_amdgcn_readfirstlane(remap_tile(blockIdx.x, 4 * p.nblk_pml, 4 * p.nblk));
    const int blk = tile >> 2, sub = tile & 3;
    const bool pml = blk < p.nblk_pml;
    const real* __restrict__ qin = static_cast<const real*>(p.q_in);
    const real* __restrict__ geo0 = static_cast<const real*>(p.geo) + static_cast<size_t>(blk) * kGeo * B + 16 * sub;
    const real* __restrict__ qt = qin + static_cast<size_t>(blk) * EHS + 16 * sub;

    // wavefront u owns field component u of the tile
    const int u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane >> 4, j = lane & 15;
    const int e = 16 * sub + j;
    const int ax = (u < 3) ? u : u - 3;
    const int bb = (ax == 2) ? 0 : ax + 1;
    const int cc = (ax == 0) ? 2 : ax - 1;
    const real* __restrict__ qe = qt + j;
    const real* __restrict__ geo = geo0 + j;
    const size_t pbase = static_cast<size_t>(p.nblk) * EHS + static_cast<size_t>(blk) * EHS + e;

    // ---- operators to LDS by direct global->LDS loads (16 bytes per lane, 1 KiB per wavefront)
    {
        const char* __restrict__ src = static_cast<const char*>(p.frags);
        char* dst = reinterpret_cast<char*>(fr);
        for (int c = u; c < NCHUNK; c += 6)
            __builtin_amdgcn_global_load_lds(src + c * 1024 + lane * 16, dst + c * 1024, 16, 0, 0);
    }
    // ---- issue every load that does not depend on the flux before the barrier
    real bf[SP], bp[SP], xb[SP], xc[SP];
    const int fo = (u < 3) ? 3 : 0;
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        const int node = 4 * s + g;
        const bool ok = (SP * 4 == Np) || node < Np;
        const int nd = ok ? node : 0;
        bf[s] = pml ? qe[(u * Np + nd) * B] : real(0);
        bp[s] = pml ? qin[pbase + static_cast<size_t>(u * Np + nd) * B] : real(0);
        xb[s] = qe[((fo + bb) * Np + nd) * B];
        xc[s] = qe[((fo + cc) * Np + nd) * B];
        if (!ok) bf[s] = bp[s] = xb[s] = xc[s] = real(0);
    }
    const real sgn = (u < 3) ? real(1) : real(-1);
    const real mrb = geo[bb * B], mrc = geo[cc * B];
    const real msb = geo[(3 + bb) * B], msc = geo[(3 + cc) * B];
    const real mtb = geo[(6 + bb) * B], mtc = geo[(6 + cc) * B];

    // ---- upwind flux of all six components at the 4 Nfp face nodes, once per tile
    {
        const int* __restrict__ nbr = p.nbr + static_cast<size_t>(blk) * NF * B + 16 * sub;
        const real alpha = static_cast<real>(p.alpha);
        real own[FIT][6], nb[FIT][6], nv[FIT][4];
        int vv[FIT];
#pragma unroll
        for (int it = 0; it < FIT; ++it) {
            const int pi0 = tid + it * kMfmaThreads;
            const int pi = pi0 < NF * 16 ? pi0 : 0;
            const int fn = pi >> 4, jj = pi & 15;
            const int fc = fn / Nfp;
            const int jn = p.fmask[fn];
#pragma unroll
            for (int c = 0; c < 6; ++c) own[it][c] = qt[(c * Np + jn) * B + jj];
            vv[it] = nbr[fn * B + jj];
#pragma unroll
            for (int c = 0; c < 4; ++c) nv[it][c] = geo0[(9 + 4 * fc + c) * B + jj];
        }
#pragma unroll
        for (int it = 0; it < FIT; ++it) {
            const int off = vv[it] >= 0 ? vv[it] : ~vv[it];
            const real* __restrict__ qp = qin + off;
#pragma unroll
            for (int c = 0; c < 6; ++c) nb[it][c] = qp[c * Np * B];
        }
#pragma unroll
        for (int it = 0; it < FIT; ++it) {
            const int pi = tid + it * kMfmaThreads;
            if (pi >= NF * 16) continue;
            const real sE = vv[it] >= 0 ? real(1) : real(-1);  // PEC wall: E+ = -E-, H+ = H-
            const real dEx = own[it][0] - sE * nb[it][0], dEy = own[it][1] - sE * nb[it][1], dEz = own[it][2] - sE * nb[it][2];
            const real dHx = own[it][3] - nb[it][3], dHy = own[it][4] - nb[it][4], dHz = own[it][5] - nb[it][5];
            const real nx = nv[it][0], ny = nv[it][1], nz = nv[it][2];
            const real hs = real(0.5) * nv[it][3];
            const real ndE = nx * dEx + ny * dEy + nz * dEz;
            const real ndH = nx * dHx + ny * dHy + nz * dHz;
            real* f = fl + pi;  // (fn * 16 + jj)
            f[0 * NF * 16] = hs * (-(ny * dHz - nz * dHy) + alpha * (nx * ndE - dEx));
            f[1 * NF * 16] = hs * (-(nz * dHx - nx * dHz) + alpha * (ny * ndE - dEy));
            f[2 * NF * 16] = hs * (-(nx * dHy - ny * dHx) + alpha * (nz * ndE - dEz));
            f[3 * NF * 16] = hs * ((ny * dEz - nz * dEy) + alpha * (nx * ndH - dHx));
            f[4 * NF * 16] = hs * ((nz * dEx - nx * dEz) + alpha * (ny * ndH - dHy));
            f[5 * NF * 16] = hs * ((nx * dEy - ny * dEx) + alpha * (nz * ndH - dHz));
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the direct loads into LDS have landed
    __syncthreads();

    const int Nq = p.Nq;
    const int SQ = (Nq + 3) / 4;
    real* __restrict__ rs = static_cast<real*>(p.res);
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    const real rkA = static_cast<real>(p.rk_a), rkB = static_cast<real>(p.rk_b), dt = static_cast<real>(p.dt);
    const bool read_res = p.read_res != 0;
    auto frag = [&](int f) -> real { return fr[f * 64 + lane]; };

    v4 R[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) R[t] = v4{0, 0, 0, 0};

    // ---- B. lift of the flux of component u (eqs. (15), (17))
#pragma unroll
    for (int s = 0; s < SF; ++s) {
        const real b = fl[(u * NF + 4 * s + g) * 16 + j];
#pragma unroll
        for (int t = 0; t < PT; ++t) R[t] = M::run(frag(OFF_L + t * SF + s), b, R[t]);
    }

    // ---- C. volume curl: +curl H (E components), -curl E (H components)
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        const real gr = sgn * (mrb * xc[s] - mrc * xb[s]);
        const real gs = sgn * (msb * xc[s] - msc * xb[s]);
        const real gt = sgn * (mtb * xc[s] - mtc * xb[s]);
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            R[t] = M::run(frag(OFF_D + (0 * PT + t) * SP + s), gr, R[t]);
            R[t] = M::run(frag(OFF_D + (1 * PT + t) * SP + s), gs, R[t]);
            R[t] = M::run(frag(OFF_D + (2 * PT + t) * SP + s), gt, R[t]);
        }
    }

    // residual and field of component u for the final update, issued before the products
    real rold[PT][4], qold[PT][4];
    {
        const size_t eb = static_cast<size_t>(blk) * EHS + e;
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                const size_t idx = eb + static_cast<size_t>(u * Np + (node < Np ? node : 0)) * B;
                rold[t][v] = read_res ? rs[idx] : real(0);
                qold[t][v] = qin[idx];
            }
    }

    // ---- A. PML terms at the cubature points (eqs. (26)-(29))
    if (pml) {
        const real* __restrict__ sg = static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + e;
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e : nullptr;
        // coefficient samples and the residual / field of the auxiliary component, issued early
        real sa[QT][4], sb[QT][4], sc[QT][4];
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 16 * t + 4 * v + g;
                const int qq = q < Nq ? q : 0;
                sa[t][v] = sg[(ax * Nq + qq) * B];
                sb[t][v] = sg[(bb * Nq + qq) * B];
                sc[t][v] = sg[(cc * Nq + qq) * B];
            }
        real rold[PT][4], qold[PT][4];
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                const size_t idx = pbase + static_cast<size_t>(u * Np + (node < Np ? node : 0)) * B;
                rold[t][v] = read_res ? rs[idx] : real(0);
                qold[t][v] = qin[idx];
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
                    real bq, cq, dq, kinv;
                    if (KAPPA) {
                        const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                        kinv = real(1) / ka;
                        const real aa = kb * kc * kinv;
                        bq = (sb[t][v] * kc + sc[t][v] * kb - aa * sa[t][v]) * kinv;
                        cq = sb[t][v] * sc[t][v] - bq * sa[t][v];
                        dq = sa[t][v] * kinv;
                    } else {
                        kinv = real(1);
                        bq = sb[t][v] + sc[t][v] - sa[t][v];
                        cq = sb[t][v] * sc[t][v] - bq * sa[t][v];
                        dq = sa[t][v];
                    }
                    const real vf = VF[t][v], vp = VP[t][v];
                    t1 = bq * vf + cq * vp;
                    t2 = kinv * vf - dq * vp;
                }
                VF[t][v] = -t1;
                VP[t][v] = t2;
            }
        // rhs_P = P_q t2 and R = -P_q t1
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
                        R[t] = M::run(a, VF[tq][v], R[t]);
                    }
                }
            }
        // LSERK update of the auxiliary component
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                if (node < Np) {
                    const size_t idx = pbase + static_cast<size_t>(u * Np + node) * B;
                    const real r = dt * RP[t][v] + rkA * rold[t][v];
                    rs[idx] = r;
                    qo[idx] = qold[t][v] + rkB * r;
                }
            }
    }

    // ---- dipole source on the electric components
    if (u < 3) {
        const int slot = p.src_slot[blk];
        if (slot >= 0) {
            const real gsrc = static_cast<real>(p.src_g);
            const real* __restrict__ S = static_cast<const real*>(p.src) + (static_cast<size_t>(slot) * 3 + u) * Np * B + e;
#pragma unroll
            for (int t = 0; t < PT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int node = 16 * t + 4 * v + g;
                    if (node < Np) R[t][v] -= gsrc * S[node * B];
                }
        }
    }

    // ---- D. weight-adjusted inverse mass on PML tiles: rhs = P_q a^-1 V_q R (eq. (21))
    if (pml) {
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
                    for (int t = 0; t < QT; ++t) Z[t] = M::run(frag(OFF_VQ + t * SP + sp), R[tp][v], Z[t]);
                }
            }
        if (KAPPA) {
            const real* __restrict__ kp = static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e;
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
        for (int t = 0; t < PT; ++t) R[t] = O[t];
    }

    // ---- LSERK4 update of component u
    {
        const size_t eb = static_cast<size_t>(blk) * EHS + e;
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                if (node < Np) {
                    const size_t idx = eb + static_cast<size_t>(u * Np + node) * B;
                    const real r = dt * R[t][v] + rkA * rold[t][v];
                    rs[idx] = r;
                    qo[idx] = qold[t][v] + rkB * r;
                }
            }
    }
}

template <typename real, int N, int QT, bool K>
int launch_t(const StageParams& p, hipStream_t s) {
    hipLaunchKernelGGL((stage_mfma_kernel<real, N, QT, K>), dim3(4 * p.nblk), dim3(kMfmaThreads), 0, s, p);
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
