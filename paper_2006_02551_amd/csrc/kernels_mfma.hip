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

// Copies nseg row segments of `seg_bytes` (16 elements of one row) into LDS
// with direct 16-byte global->LDS loads, 1 KiB per wavefront instruction.
// Segment k of the destination is segment k of the source list, whose global
// address is base + k * stride_bytes.  Waves w, w+nw, ... take 1 KiB chunks.
__device__ __forceinline__ void stage_rows(const char* __restrict__ base, size_t stride_bytes, int seg_bytes,
                                           int nseg, char* lds, int wave, int nw, int lane) {
    const int total = nseg * seg_bytes;
    const int nchunk = (total + 1023) / 1024;
    for (int c = wave; c < nchunk; c += nw) {
        int byte = c * 1024 + lane * 16;
        if (byte >= total) byte = total - 16;  // stays inside the source rows; lands in LDS padding
        const int seg = byte / seg_bytes, off = byte - seg * seg_bytes;
        __builtin_amdgcn_global_load_lds(base + seg * stride_bytes + off, lds + c * 1024, 16, 0, 0);
    }
}

constexpr int pad1k(int bytes) { return (bytes + 1023) / 1024 * 1024; }

template <typename real, int N, int QT, bool KAPPA>
__global__ __launch_bounds__(kMfmaThreads) void stage_mfma_kernel(StageParams p) {
    using M = Mma<real>;
    using v4 = typename M::v4;
    constexpr int Np = Ord<N>::Np, Nfp = Ord<N>::Nfp, B = kBlock, T = 16;
    constexpr int NF = 4 * Nfp;         // face nodes per element
    constexpr int PT = (Np + 15) / 16;  // node tiles
    constexpr int SP = (Np + 3) / 4;    // k-steps over nodes
    constexpr int SQM = 4 * QT;         // k-steps reserved over cubature points
    constexpr int SF = Nfp;             // k-steps over the face nodes
    constexpr int QMAX = 16 * QT;       // cubature points the sigma staging can hold
    constexpr int OFF_VQ = 0;
    constexpr int OFF_PQ = OFF_VQ + QT * SP;
    constexpr int OFF_D = OFF_PQ + PT * SQM;
    constexpr int OFF_L = OFF_D + 3 * PT * SP;
    constexpr int NFRAG = OFF_L + PT * SF;
    constexpr int EHS = 6 * Np * B;
    constexpr int FIT = (NF * T + kMfmaThreads - 1) / kMfmaThreads;  // flux items per thread
    constexpr int RB = static_cast<int>(sizeof(real));
    // LDS: operator fragments, the tile's E,H rows, sigma rows, geometry rows,
    // neighbour offsets, and the flux (all padded to whole KiB for the staging copies)
    constexpr int L_FR = pad1k(NFRAG * 64 * RB);
    constexpr int L_EH = pad1k(6 * Np * T * RB);
    constexpr int L_SG = pad1k(3 * QMAX * T * RB);
    constexpr int L_GE = pad1k(kGeo * T * RB);
    constexpr int L_NB = pad1k(NF * T * 4);
    __shared__ __attribute__((aligned(16))) char smem[L_FR + L_EH + L_SG + L_GE + L_NB];
    __shared__ real fl[6 * NF * T];  // flux [component][face node][element of the tile]
    real* fr = reinterpret_cast<real*>(smem);
    real* eh = reinterpret_cast<real*>(smem + L_FR);
    real* sgs = reinterpret_cast<real*>(smem + L_FR + L_EH);
    real* ges = reinterpret_cast<real*>(smem + L_FR + L_EH + L_SG);
    int* nbs = reinterpret_cast<int*>(smem + L_FR + L_EH + L_SG + L_GE);

    const int tid = static_cast<int>(threadIdx.x);
    const int tile = __builtin_amdgcn_readfirstlane(remap_tile(blockIdx.x, 4 * p.nblk_pml, 4 * p.nblk));
    const int blk = tile >> 2, sub = tile & 3;
    const bool pml = blk < p.nblk_pml;
    const int Nq = p.Nq;
    const int u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane >> 4, j = lane & 15;
    const int e = T * sub + j;
    const real* __restrict__ qin = static_cast<const real*>(p.q_in);

    // ---- stage the tile into LDS (direct global->LDS loads)
    {
        const size_t row = static_cast<size_t>(B) * RB;  // bytes between rows of the blocked layout
        stage_rows(reinterpret_cast<const char*>(p.frags), 1024, 1024, NFRAG * 64 * RB / 1024 + ((NFRAG * 64 * RB) % 1024 ? 1 : 0),
                   smem, u, 6, lane);
        stage_rows(reinterpret_cast<const char*>(qin + static_cast<size_t>(blk) * EHS + T * sub), row, T * RB, 6 * Np,
                   smem + L_FR, u, 6, lane);
        stage_rows(reinterpret_cast<const char*>(static_cast<const real*>(p.geo) + static_cast<size_t>(blk) * kGeo * B + T * sub),
                   row, T * RB, kGeo, smem + L_FR + L_EH + L_SG, u, 6, lane);
        stage_rows(reinterpret_cast<const char*>(p.nbr + static_cast<size_t>(blk) * NF * B + T * sub), static_cast<size_t>(B) * 4,
                   T * 4, NF, smem + L_FR + L_EH + L_SG + L_GE, u, 6, lane);
        if (pml)
            stage_rows(reinterpret_cast<const char*>(static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + T * sub),
                       row, T * RB, 3 * Nq, smem + L_FR + L_EH, u, 6, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- per-wave loads that only this wave needs, issued to overlap the flux phase
    const size_t pbase = static_cast<size_t>(p.nblk) * EHS + static_cast<size_t>(blk) * EHS + e;
    const size_t ebase = static_cast<size_t>(blk) * EHS + e;
    real* __restrict__ rs = static_cast<real*>(p.res);
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    const bool read_res = p.read_res != 0;
    real bp[SP];
    real rP[PT][4], qP[PT][4], rE[PT][4];
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        const int node = 4 * s + g;
        const int nd = ((SP * 4 == Np) || node < Np) ? node : 0;
        bp[s] = pml ? qin[pbase + static_cast<size_t>(u * Np + nd) * B] : real(0);
    }
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int node = 16 * t + 4 * v + g;
            const int nd = node < Np ? node : 0;
            rP[t][v] = (pml && read_res) ? rs[pbase + static_cast<size_t>(u * Np + nd) * B] : real(0);
            qP[t][v] = pml ? qin[pbase + static_cast<size_t>(u * Np + nd) * B] : real(0);
            rE[t][v] = read_res ? rs[ebase + static_cast<size_t>(u * Np + nd) * B] : real(0);
        }

    // ---- upwind flux of all six components at the 4 Nfp face nodes, once per tile
    {
        const real alpha = static_cast<real>(p.alpha);
        real nb[FIT][6];
        int vv[FIT];
#pragma unroll
        for (int it = 0; it < FIT; ++it) {
            const int pi0 = tid + it * kMfmaThreads;
            const int pi = pi0 < NF * T ? pi0 : 0;
            vv[it] = nbs[pi];  // [face node][element]
            const int off = vv[it] >= 0 ? vv[it] : ~vv[it];
            const real* __restrict__ qp = qin + off;
#pragma unroll
            for (int c = 0; c < 6; ++c) nb[it][c] = qp[c * Np * B];
        }
#pragma unroll
        for (int it = 0; it < FIT; ++it) {
            const int pi = tid + it * kMfmaThreads;
            if (pi >= NF * T) continue;
            const int fn = pi >> 4, jj = pi & 15;
            const int fc = fn / Nfp;
            const int jn = p.fmask[fn];
            const real sE = vv[it] >= 0 ? real(1) : real(-1);  // PEC wall: E+ = -E-, H+ = H-
            const real dEx = eh[(0 * Np + jn) * T + jj] - sE * nb[it][0];
            const real dEy = eh[(1 * Np + jn) * T + jj] - sE * nb[it][1];
            const real dEz = eh[(2 * Np + jn) * T + jj] - sE * nb[it][2];
            const real dHx = eh[(3 * Np + jn) * T + jj] - nb[it][3];
            const real dHy = eh[(4 * Np + jn) * T + jj] - nb[it][4];
            const real dHz = eh[(5 * Np + jn) * T + jj] - nb[it][5];
            const real nx = ges[(9 + 4 * fc) * T + jj], ny = ges[(10 + 4 * fc) * T + jj], nz = ges[(11 + 4 * fc) * T + jj];
            const real hs = real(0.5) * ges[(12 + 4 * fc) * T + jj];
            const real ndE = nx * dEx + ny * dEy + nz * dEz;
            const real ndH = nx * dHx + ny * dHy + nz * dHz;
            real* f = fl + pi;
            f[0 * NF * T] = hs * (-(ny * dHz - nz * dHy) + alpha * (nx * ndE - dEx));
            f[1 * NF * T] = hs * (-(nz * dHx - nx * dHz) + alpha * (ny * ndE - dEy));
            f[2 * NF * T] = hs * (-(nx * dHy - ny * dHx) + alpha * (nz * ndE - dEz));
            f[3 * NF * T] = hs * ((ny * dEz - nz * dEy) + alpha * (nx * ndH - dHx));
            f[4 * NF * T] = hs * ((nz * dEx - nx * dEz) + alpha * (ny * ndH - dHy));
            f[5 * NF * T] = hs * ((nx * dEy - ny * dEx) + alpha * (nz * ndH - dHz));
        }
    }
    __syncthreads();

    const int SQ = (Nq + 3) / 4;
    const int ax = (u < 3) ? u : u - 3;
    const int bb = (ax == 2) ? 0 : ax + 1;
    const int cc = (ax == 0) ? 2 : ax - 1;
    const real rkA = static_cast<real>(p.rk_a), rkB = static_cast<real>(p.rk_b), dt = static_cast<real>(p.dt);
    auto frag = [&](int f) -> real { return fr[f * 64 + lane]; };
    auto ehv = [&](int c, int node) -> real { return eh[(c * Np + node) * T + j]; };

    v4 R[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) R[t] = v4{0, 0, 0, 0};

    // ---- B. lift of the flux of component u (eqs. (15), (17))
#pragma unroll
    for (int s = 0; s < SF; ++s) {
        const real b = fl[(u * NF + 4 * s + g) * T + j];
#pragma unroll
        for (int t = 0; t < PT; ++t) R[t] = M::run(frag(OFF_L + t * SF + s), b, R[t]);
    }

    // ---- C. volume curl: +curl H (E components), -curl E (H components)
    {
        const int fo = (u < 3) ? 3 : 0;
        const real sgn = (u < 3) ? real(1) : real(-1);
        const real rb = sgn * ges[bb * T + j], rc = sgn * ges[cc * T + j];
        const real sb = sgn * ges[(3 + bb) * T + j], sc = sgn * ges[(3 + cc) * T + j];
        const real tb = sgn * ges[(6 + bb) * T + j], tc = sgn * ges[(6 + cc) * T + j];
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const int node = 4 * s + g;
            const bool ok = (SP * 4 == Np) || node < Np;
            const real xb = ok ? ehv(fo + bb, node) : real(0);
            const real xc = ok ? ehv(fo + cc, node) : real(0);
            const real gr = rb * xc - rc * xb, gs = sb * xc - sc * xb, gt = tb * xc - tc * xb;
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                R[t] = M::run(frag(OFF_D + (0 * PT + t) * SP + s), gr, R[t]);
                R[t] = M::run(frag(OFF_D + (1 * PT + t) * SP + s), gs, R[t]);
                R[t] = M::run(frag(OFF_D + (2 * PT + t) * SP + s), gt, R[t]);
            }
        }
    }

    // ---- A. PML terms at the cubature points (eqs. (26)-(29))
    if (pml) {
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e : nullptr;
        v4 VF[QT], VP[QT];
#pragma unroll
        for (int t = 0; t < QT; ++t) VF[t] = VP[t] = v4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            const int node = 4 * s + g;
            const bool ok = (SP * 4 == Np) || node < Np;
            const real bf = ok ? ehv(u, node) : real(0);
            const real bpv = ok ? bp[s] : real(0);
#pragma unroll
            for (int t = 0; t < QT; ++t) {
                const real a = frag(OFF_VQ + t * SP + s);
                VF[t] = M::run(a, bf, VF[t]);
                VP[t] = M::run(a, bpv, VP[t]);
            }
        }
        // eq. (9) at cubature point q = 16 t + 4 v + g: VF <- -t1, VP <- t2
#pragma unroll
        for (int t = 0; t < QT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 16 * t + 4 * v + g;
                real t1 = real(0), t2 = real(0);
                if (q < Nq) {
                    const real sa = sgs[(ax * Nq + q) * T + j], sbq = sgs[(bb * Nq + q) * T + j], scq = sgs[(cc * Nq + q) * T + j];
                    real bq, cq, dq, kinv;
                    if (KAPPA) {
                        const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                        kinv = real(1) / ka;
                        const real aa = kb * kc * kinv;
                        bq = (sbq * kc + scq * kb - aa * sa) * kinv;
                        cq = sbq * scq - bq * sa;
                        dq = sa * kinv;
                    } else {
                        kinv = real(1);
                        bq = sbq + scq - sa;
                        cq = sbq * scq - bq * sa;
                        dq = sa;
                    }
                    const real vf = VF[t][v], vp = VP[t][v];
                    t1 = bq * vf + cq * vp;
                    t2 = kinv * vf - dq * vp;
                }
                VF[t][v] = -t1;
                VP[t][v] = t2;
            }
        // rhs_P = P_q t2 and R -= P_q t1
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
                    const real r = dt * RP[t][v] + rkA * rP[t][v];
                    rs[idx] = r;
                    qo[idx] = qP[t][v] + rkB * r;
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
#pragma unroll
    for (int t = 0; t < PT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int node = 16 * t + 4 * v + g;
            if (node < Np) {
                const size_t idx = ebase + static_cast<size_t>(u * Np + node) * B;
                const real r = dt * R[t][v] + rkA * rE[t][v];
                rs[idx] = r;
                qo[idx] = ehv(u, node) + rkB * r;
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

// Order / cubature-tile combinations with a matrix-core kernel.  FP64 at
// N = 4 would need more than the 160 KiB of LDS of a compute unit.
template <typename real>
int launch_r(int N, int QT, bool k, const StageParams& p, hipStream_t s) {
    switch (N * 10 + QT) {
        case 11: return launch_k<real, 1, 1>(k, p, s);
        case 12: return launch_k<real, 1, 2>(k, p, s);
        case 21: return launch_k<real, 2, 1>(k, p, s);
        case 22: return launch_k<real, 2, 2>(k, p, s);
        case 32: return launch_k<real, 3, 2>(k, p, s);
        case 33: return launch_k<real, 3, 3>(k, p, s);
        default: return -1;
    }
}

int launch_r4(int QT, bool k, const StageParams& p, hipStream_t s) {
    switch (QT) {
        case 3: return launch_k<float, 4, 3>(k, p, s);
        case 4: return launch_k<float, 4, 4>(k, p, s);
        default: return -1;
    }
}

}  // namespace

bool mfma_supported(int N, int Nq, int precision) {
    const int QT = (Nq + 15) / 16;
    switch (N * 10 + QT) {
        case 11: case 12: case 21: case 22: case 32: case 33: return true;
        case 43: case 44: return precision != 0;
        default: return false;
    }
}

int launch_stage_mfma(int precision, int N, bool has_kappa, const StageParams& p, hipStream_t s) {
    const int QT = (p.Nq + 15) / 16;
    if (precision == 0) return launch_r<double>(N, QT, has_kappa, p, s);
    if (N == 4) return launch_r4(QT, has_kappa, p, s);
    return launch_r<float>(N, QT, has_kappa, p, s);
}

}  // namespace wdg
