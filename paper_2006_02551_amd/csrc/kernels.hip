// HIP kernels for gfx950: the fused per-stage right-hand side of eqs. (26)-(29)
// with the LSERK4 update, plus the FP64 probe and energy readouts.
//
// Work decomposition of the stage kernel.  A workgroup owns one block of 64
// element slots of one class (PML or interior) and has six wavefronts; wave u
// owns Cartesian field component u (Ex, Ey, Ez, Hx, Hy, Hz) and lane e owns
// element slot e.  Every reference operator entry a lane needs is therefore
// the same across the wavefront, so it is read with scalar loads and enters
// the FMA as a scalar operand, and every field load is a coalesced 64-wide
// row of the blocked layout.  The only cross-wave exchange is the face flux,
// staged through LDS one face at a time.
//
// Per stage and component u of field f with auxiliary field P (PML blocks):
//   1. t1 = b V_q f + c V_q P,  t2 = kappa^{-1} V_q f - d V_q P  (eq. (9) entries
//      formed in registers from sigma (and kappa) at the cubature points),
//      rhs_P = P_q t2,  w = -P_q t1                            (eqs. (26)-(29))
//   2. w += LIFT (Fscale * upwind flux)                        (eqs. (15), (17))
//   3. w += curl via D_r, D_s, D_t and the metric terms        (eqs. (15)-(16))
//   4. w -= J (dipole source, electric components)
//   5. rhs_f = P_q a^{-1} V_q w       (weight-adjusted inverse mass, eq. (21))
//   6. res = A res + dt rhs;  q_out = q_in + B res             (LSERK4)
// Interior blocks skip 1 and 5 (rhs_f = w, no auxiliary fields).
//
// The same kernel evaluates two other PML schemes for comparison:
// * direct (stored matrices, eqs. (10)-(15) with exact weighted mass
//   matrices): on PML blocks this kernel stops after 4 and writes w (the
//   vacuum right-hand side) to a work buffer; direct_apply_kernel then
//   streams the five per-element N_p x N_p products of the layout in
//   device.hpp (15 N_p^2 words per element) and finishes 5 and 6:
//     rhs_f = G_1 w - G_2 f - G_3 P,   rhs_P = G_4 f - G_5 P;
// * element-constant coefficients (one sigma_u, kappa_u per element):
//   the weighted mass matrices are multiples of M_k, so 1 and 5 are
//   pointwise: w = -(b f + c P), rhs_P = f / kappa - d P, rhs_f = w / a.
#include "device.hpp"

namespace wdg {
namespace {

template <int N>
struct Ord {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup id mod 8).
// Map them so that every XCD walks a contiguous, spatially coherent run of
// blocks inside each class (remap_range); neighbour traces then tend to hit its own L2.

template <typename real, int N, bool KAPPA, int MODE>
__global__ __launch_bounds__(kThreads) void stage_kernel(StageParams p) {
    constexpr int Np = Ord<N>::Np, Nfp = Ord<N>::Nfp, B = kBlock;
    constexpr int EHS = 6 * Np * B;  // E,H words per block
    __shared__ real Fl[6 * Nfp * B];

    const int u = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / B);
    const int lane = static_cast<int>(threadIdx.x) % B;
    const int bid = p.order_rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x);
    const int blk = __builtin_amdgcn_readfirstlane(remap_range(bid, p.pml0, p.npml, p.int0, p.nint));
    const bool pml = blk < p.nblk_pml;
    const int Nq = p.Nq;

    const real* __restrict__ qin = static_cast<const real*>(p.q_in);
    const real* __restrict__ qe = qin + static_cast<size_t>(blk) * EHS + lane;
    const real* __restrict__ geo = static_cast<const real*>(p.geo) + static_cast<size_t>(blk) * kGeo * B + lane;
    const real* __restrict__ DrT = static_cast<const real*>(p.DrT);
    const real* __restrict__ DsT = static_cast<const real*>(p.DsT);
    const real* __restrict__ DtT = static_cast<const real*>(p.DtT);
    const real* __restrict__ LIFTT = static_cast<const real*>(p.LIFTT);
    const real* __restrict__ Vq = static_cast<const real*>(p.Vq);
    const real* __restrict__ PqT = static_cast<const real*>(p.PqT);

    // (ax, bb, cc) is the cyclic triple (u, v, w) of eq. (9) for this component.
    const int ax = (u < 3) ? u : u - 3;
    const int bb = (ax == 2) ? 0 : ax + 1;
    const int cc = (ax == 0) ? 2 : ax - 1;
    const size_t pbase = static_cast<size_t>(p.nblk) * EHS + static_cast<size_t>(blk) * EHS + lane;

    real w[Np];      // bracket of eqs. (26)-(27), then rhs of f
    real rhsP[Np];   // rhs of the auxiliary field
    real f[Np], P[Np];  // own field component and its auxiliary field (PML blocks)
    real ainv = real(1);  // element-constant scheme: 1 / a_uu

    // ---- 1. PML terms
    if (pml && MODE != kPmlDirect) {
#pragma unroll
        for (int j = 0; j < Np; ++j) {
            f[j] = qe[(u * Np + j) * B];
            P[j] = qin[pbase + (u * Np + j) * B];
            w[j] = real(0);
            rhsP[j] = real(0);
        }
    }
    if (pml && MODE == kPmlConstant) {
        // eq. (9) at the element's constant sigma, kappa
        const real* __restrict__ ec = static_cast<const real*>(p.pml_mats) + static_cast<size_t>(blk) * 6 * B + lane;
        const real sa = ec[ax * B], sb = ec[bb * B], sc = ec[cc * B];
        const real ka = ec[(3 + ax) * B], kb = ec[(3 + bb) * B], kc = ec[(3 + cc) * B];
        const real kinv = real(1) / ka;
        const real a = kb * kc * kinv;
        const real bq = (sb * kc + sc * kb - a * sa) * kinv;
        const real cq = sb * sc - bq * sa;
        const real dq = sa * kinv;
        ainv = ka / (kb * kc);
#pragma unroll
        for (int j = 0; j < Np; ++j) {
            w[j] = -(bq * f[j] + cq * P[j]);
            rhsP[j] = kinv * f[j] - dq * P[j];
        }
    }
    if (pml && MODE == kPmlWaa) {
        const real* __restrict__ sg = static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + lane;
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + lane : nullptr;
        for (int q = 0; q < Nq; ++q) {
            real vf = real(0), vp = real(0);
#pragma unroll
            for (int j = 0; j < Np; ++j) {
                const real v = Vq[q * Np + j];
                vf += v * f[j];
                vp += v * P[j];
            }
            const real sa = sg[(ax * Nq + q) * B], sb = sg[(bb * Nq + q) * B], sc = sg[(cc * Nq + q) * B];
            real bq, cq, dq, kinv;
            if (KAPPA) {
                const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                kinv = real(1) / ka;
                const real a = kb * kc * kinv;
                bq = (sb * kc + sc * kb - a * sa) * kinv;
                cq = sb * sc - bq * sa;
                dq = sa * kinv;
            } else {
                kinv = real(1);
                bq = sb + sc - sa;
                cq = sb * sc - bq * sa;
                dq = sa;
            }
            const real t1 = bq * vf + cq * vp;
            const real t2 = kinv * vf - dq * vp;
#pragma unroll
            for (int i = 0; i < Np; ++i) {
                const real pw = PqT[q * Np + i];
                w[i] -= pw * t1;
                rhsP[i] += pw * t2;
            }
        }
    }
    if (!pml || MODE == kPmlDirect) {
#pragma unroll
        for (int i = 0; i < Np; ++i) w[i] = real(0);
    }

    // ---- 2. surface term: upwind flux lifted face by face
    const int* __restrict__ nbr = p.nbr + static_cast<size_t>(blk) * 4 * Nfp * B + lane;
    const real alpha = static_cast<real>(p.alpha);
    for (int fc = 0; fc < 4; ++fc) {
        for (int m = u; m < Nfp; m += 6) {
            const int jn = p.fmask[fc * Nfp + m];
            const real Ex = qe[(0 * Np + jn) * B], Ey = qe[(1 * Np + jn) * B], Ez = qe[(2 * Np + jn) * B];
            const real Hx = qe[(3 * Np + jn) * B], Hy = qe[(4 * Np + jn) * B], Hz = qe[(5 * Np + jn) * B];
            const int v = nbr[(fc * Nfp + m) * B];
            const int off = v >= 0 ? v : ~v;
            const real sE = v >= 0 ? real(1) : real(-1);  // PEC wall: E+ = -E-, H+ = H-
            const real* __restrict__ qp = qin + off;
            const real dEx = Ex - sE * qp[0 * Np * B], dEy = Ey - sE * qp[1 * Np * B], dEz = Ez - sE * qp[2 * Np * B];
            const real dHx = Hx - qp[3 * Np * B], dHy = Hy - qp[4 * Np * B], dHz = Hz - qp[5 * Np * B];
            const real nx = geo[(9 + 4 * fc) * B], ny = geo[(10 + 4 * fc) * B], nz = geo[(11 + 4 * fc) * B];
            const real hs = real(0.5) * geo[(12 + 4 * fc) * B];
            const real ndE = nx * dEx + ny * dEy + nz * dEz;
            const real ndH = nx * dHx + ny * dHy + nz * dHz;
            real* fl = Fl + m * B + lane;
            fl[0 * Nfp * B] = hs * (-(ny * dHz - nz * dHy) + alpha * (nx * ndE - dEx));
            fl[1 * Nfp * B] = hs * (-(nz * dHx - nx * dHz) + alpha * (ny * ndE - dEy));
            fl[2 * Nfp * B] = hs * (-(nx * dHy - ny * dHx) + alpha * (nz * ndE - dEz));
            fl[3 * Nfp * B] = hs * ((ny * dEz - nz * dEy) + alpha * (nx * ndH - dHx));
            fl[4 * Nfp * B] = hs * ((nz * dEx - nx * dEz) + alpha * (ny * ndH - dHy));
            fl[5 * Nfp * B] = hs * ((nx * dEy - ny * dEx) + alpha * (nz * ndH - dHz));
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < Nfp; ++m) {
            const real fv = Fl[(u * Nfp + m) * B + lane];
#pragma unroll
            for (int i = 0; i < Np; ++i) w[i] += LIFTT[(fc * Nfp + m) * Np + i] * fv;
        }
        __syncthreads();
    }

    // ---- 3. volume curl: +curl H for E components, -curl E for H components
    {
        const int fo = (u < 3) ? 3 : 0;
        const real sgn = (u < 3) ? real(1) : real(-1);
        const real rb = sgn * geo[bb * B], rc = sgn * geo[cc * B];
        const real sb = sgn * geo[(3 + bb) * B], sc = sgn * geo[(3 + cc) * B];
        const real tb = sgn * geo[(6 + bb) * B], tc = sgn * geo[(6 + cc) * B];
        const real* __restrict__ Fb = qe + (fo + bb) * Np * B;
        const real* __restrict__ Fc = qe + (fo + cc) * Np * B;
#pragma unroll 4
        for (int j = 0; j < Np; ++j) {
            const real xb = Fb[j * B], xc = Fc[j * B];
            const real gr = rb * xc - rc * xb, gs = sb * xc - sc * xb, gt = tb * xc - tc * xb;
#pragma unroll
            for (int i = 0; i < Np; ++i) w[i] += DrT[j * Np + i] * gr + DsT[j * Np + i] * gs + DtT[j * Np + i] * gt;
        }
    }

    // ---- 4. dipole source on the electric components
    if (u < 3) {
        const int slot = p.src_slot[blk];
        if (slot >= 0) {
            const real* __restrict__ S = static_cast<const real*>(p.src) + (static_cast<size_t>(slot) * 3 + u) * Np * B + lane;
            const real gs = static_cast<real>(p.src_g);
#pragma unroll
            for (int i = 0; i < Np; ++i) w[i] -= gs * S[i * B];
        }
    }

    if (MODE == kPmlDirect && pml) {
        // the direct scheme's PML terms and update follow in direct_apply_kernel
        real* __restrict__ wo = static_cast<real*>(p.pml_work) + (static_cast<size_t>(blk) * 6 + u) * Np * B + lane;
#pragma unroll
        for (int i = 0; i < Np; ++i) wo[i * B] = w[i];
        return;
    }

    // ---- 5. weight-adjusted inverse mass: rhs_f = P_q a^{-1} V_q w
    if (pml && MODE == kPmlConstant) {
#pragma unroll
        for (int i = 0; i < Np; ++i) w[i] *= ainv;
    }
    if (pml && MODE == kPmlWaa && (KAPPA || !p.waa_skip)) {  // skipped only on request where it is the identity
        real rf[Np];
#pragma unroll
        for (int i = 0; i < Np; ++i) rf[i] = real(0);
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + lane : nullptr;
        for (int q = 0; q < Nq; ++q) {
            real z = real(0);
#pragma unroll
            for (int j = 0; j < Np; ++j) z += Vq[q * Np + j] * w[j];
            if (KAPPA) {
                const real ka = kp[(ax * Nq + q) * B], kb = kp[(bb * Nq + q) * B], kc = kp[(cc * Nq + q) * B];
                z *= ka / (kb * kc);
            }
#pragma unroll
            for (int i = 0; i < Np; ++i) rf[i] += PqT[q * Np + i] * z;
        }
#pragma unroll
        for (int i = 0; i < Np; ++i) w[i] = rf[i];
    }

    // ---- 6. LSERK4 stage update
    real* __restrict__ rs = static_cast<real*>(p.res);
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    const real A = static_cast<real>(p.rk_a), Bk = static_cast<real>(p.rk_b);
    // time step of this lane's element (a per-element scale lets independent simulations share a launch)
    const real dt = static_cast<real>(p.dt_scale ? p.dt * p.dt_scale[static_cast<size_t>(blk) * B + lane] : p.dt);
    {
        const size_t eb = static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + lane;
#pragma unroll
        for (int i = 0; i < Np; ++i) {
            const size_t idx = eb + static_cast<size_t>(i) * B;
            real r = dt * w[i];
            if (p.read_res) r += A * rs[idx];
            rs[idx] = r;
            qo[idx] = qin[idx] + Bk * r;
        }
    }
    if (pml) {
        const size_t eb = pbase + static_cast<size_t>(u) * Np * B;
#pragma unroll
        for (int i = 0; i < Np; ++i) {
            const size_t idx = eb + static_cast<size_t>(i) * B;
            real r = dt * rhsP[i];
            if (p.read_res) r += A * rs[idx];
            rs[idx] = r;
            qo[idx] = qin[idx] + Bk * r;
        }
    }
}

// Direct scheme, PML terms and Runge-Kutta update of one (PML block, axis u):
// the six vectors E_u, H_u, P^E_u, P^H_u, w_E, w_H of the block's 64 elements
// are staged in LDS; wave v then takes output rows i = v, v + W, ... and, per
// row, reads the five stored rows G_m[i][:] once (64-lane coalesced) for both
// fields, so every matrix word crosses HBM once per stage.
constexpr int kApplyWaves = 8;

template <typename real, int N>
__global__ __launch_bounds__(kApplyWaves * 64) void direct_apply_kernel(StageParams p) {
    constexpr int Np = Ord<N>::Np, B = kBlock;
    constexpr int EHS = 6 * Np * B;
    constexpr size_t MS = static_cast<size_t>(Np) * Np * B;  // one stored matrix
    __shared__ real xs[6][Np][B];  // E_u, H_u, PE_u, PH_u, w_E, w_H

    const int bid = p.order_rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x);
    const int blk = p.pml0 + bid / 3, ax = bid % 3;
    const int tid = static_cast<int>(threadIdx.x);
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    const real* __restrict__ qin = static_cast<const real*>(p.q_in);
    const real* __restrict__ wk = static_cast<const real*>(p.pml_work);
    const size_t eh = static_cast<size_t>(blk) * EHS;                                 // E,H part of the block
    const size_t ph = static_cast<size_t>(p.nblk) * EHS + static_cast<size_t>(blk) * EHS;  // auxiliary part
    for (int e = tid; e < 6 * Np * B; e += kApplyWaves * 64) {
        const int v = e / (Np * B), r = e % (Np * B);
        size_t src;
        const real* base = qin;
        switch (v) {
            case 0: src = eh + static_cast<size_t>(ax) * Np * B; break;
            case 1: src = eh + static_cast<size_t>(3 + ax) * Np * B; break;
            case 2: src = ph + static_cast<size_t>(ax) * Np * B; break;
            case 3: src = ph + static_cast<size_t>(3 + ax) * Np * B; break;
            case 4: src = (static_cast<size_t>(blk) * 6 + ax) * Np * B; base = wk; break;
            default: src = (static_cast<size_t>(blk) * 6 + 3 + ax) * Np * B; base = wk; break;
        }
        (&xs[v][0][0])[r] = base[src + r];
    }
    __syncthreads();

    const real* __restrict__ G =
        static_cast<const real*>(p.pml_mats) + (static_cast<size_t>(blk) * 3 + ax) * kDirectMats * MS + lane;
    real* __restrict__ rs = static_cast<real*>(p.res);
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    const real A = static_cast<real>(p.rk_a), Bk = static_cast<real>(p.rk_b);
    const real dt = static_cast<real>(p.dt_scale ? p.dt * p.dt_scale[static_cast<size_t>(blk) * B + lane] : p.dt);
    for (int i = wave; i < Np; i += kApplyWaves) {
        const real* __restrict__ g = G + static_cast<size_t>(i) * Np * B;
        real fE = real(0), fH = real(0), pE = real(0), pH = real(0);
        // a partial unroll keeps 20 row loads in flight per wave at a modest register count
#pragma unroll 4
        for (int j = 0; j < Np; ++j) {
            const real g1 = g[j * B], g2 = g[MS + j * B], g3 = g[2 * MS + j * B];
            const real g4 = g[3 * MS + j * B], g5 = g[4 * MS + j * B];
            const real e = xs[0][j][lane], h = xs[1][j][lane], pe = xs[2][j][lane], phv = xs[3][j][lane];
            fE += g1 * xs[4][j][lane] - g2 * e - g3 * pe;
            fH += g1 * xs[5][j][lane] - g2 * h - g3 * phv;
            pE += g4 * e - g5 * pe;
            pH += g4 * h - g5 * phv;
        }
        const real out[4] = {fE, fH, pE, pH};
        const size_t idx[4] = {eh + (static_cast<size_t>(ax) * Np + i) * B + lane,
                               eh + (static_cast<size_t>(3 + ax) * Np + i) * B + lane,
                               ph + (static_cast<size_t>(ax) * Np + i) * B + lane,
                               ph + (static_cast<size_t>(3 + ax) * Np + i) * B + lane};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            real r = dt * out[c];
            if (p.read_res) r += A * rs[idx[c]];
            rs[idx[c]] = r;
            qo[idx[c]] = xs[c][i][lane] + Bk * r;
        }
    }
}

template <typename real, int N>
__global__ void probe_kernel(ProbeParams p) {
    constexpr int Np = Ord<N>::Np, B = kBlock;
    const int t = static_cast<int>(threadIdx.x);
    if (t >= p.n * 6) return;
    const int pr = t / 6, c = t % 6;
    const int slot = p.slot[pr];
    const int blk = slot / B, lane = slot % B;
    const real* q = static_cast<const real*>(p.q) + static_cast<size_t>(blk) * 6 * Np * B + static_cast<size_t>(c) * Np * B + lane;
    double v = 0.0;
    for (int i = 0; i < Np; ++i) v += p.w[pr * Np + i] * static_cast<double>(q[i * B]);
    p.out[pr * 6 + c] = v;
}

// Deterministic two-pass FP64 energy: per-block partial sums, then one block.
template <typename real, int N>
__global__ __launch_bounds__(kThreads) void energy_kernel(EnergyParams p) {
    constexpr int Np = Ord<N>::Np, B = kBlock;
    __shared__ double red[kThreads];
    const int u = static_cast<int>(threadIdx.x) / B, lane = static_cast<int>(threadIdx.x) % B;
    const int blk = blockIdx.x;
    const real* q = static_cast<const real*>(p.q) + static_cast<size_t>(blk) * 6 * Np * B + static_cast<size_t>(u) * Np * B + lane;
    double x[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) x[i] = static_cast<double>(q[i * B]);
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < Np; ++i) {
        double mi = 0.0;
#pragma unroll
        for (int j = 0; j < Np; ++j) mi += p.M[i * Np + j] * x[j];
        e += x[i] * mi;
    }
    red[threadIdx.x] = 0.5 * p.J[static_cast<size_t>(blk) * B + lane] * e;
    __syncthreads();
    for (int s = kThreads / 2; s >= 3; s /= 2) {  // 192, 96, 48, 24, 12, 6, 3
        if (static_cast<int>(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) p.partial[blk] = red[0] + red[1] + red[2];
}

__global__ __launch_bounds__(256) void sum_kernel(const double* partial, int n, double* out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = static_cast<int>(threadIdx.x); i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k /= 2) {
        if (static_cast<int>(threadIdx.x) < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <typename real, int N, bool KAPPA, int MODE>
int launch_stage_t(const StageParams& p, hipStream_t s) {
    if (p.npml + p.nint == 0) return 0;
    hipLaunchKernelGGL((stage_kernel<real, N, KAPPA, MODE>), dim3(p.npml + p.nint), dim3(kThreads), 0, s, p);
    return static_cast<int>(hipGetLastError());
}

template <typename real, int N>
int launch_apply(const StageParams& p, hipStream_t s) {
    if (p.nblk_pml == 0) return 0;
    if (p.npml == 0) return 0;
    hipLaunchKernelGGL((direct_apply_kernel<real, N>), dim3(3 * p.npml), dim3(kApplyWaves * 64), 0, s, p);
    return static_cast<int>(hipGetLastError());
}

template <typename real, int N>
int launch_direct(const StageParams& p, hipStream_t s) {
    const int e = launch_stage_t<real, N, false, kPmlDirect>(p, s);
    return e != 0 ? e : launch_apply<real, N>(p, s);
}

template <typename real, int N>
int launch_stage_n(bool k, int mode, const StageParams& p, hipStream_t s) {
    switch (mode) {
        case kPmlWaa: return k ? launch_stage_t<real, N, true, kPmlWaa>(p, s) : launch_stage_t<real, N, false, kPmlWaa>(p, s);
        case kPmlDirect: return launch_direct<real, N>(p, s);
        case kPmlConstant: return launch_stage_t<real, N, false, kPmlConstant>(p, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

template <typename real>
int launch_stage_r(int N, bool k, int mode, const StageParams& p, hipStream_t s) {
    switch (N) {
        case 1: return launch_stage_n<real, 1>(k, mode, p, s);
        case 2: return launch_stage_n<real, 2>(k, mode, p, s);
        case 3: return launch_stage_n<real, 3>(k, mode, p, s);
        case 4: return launch_stage_n<real, 4>(k, mode, p, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

template <typename real, int N>
int launch_probe_t(const ProbeParams& p, hipStream_t s) {
    hipLaunchKernelGGL((probe_kernel<real, N>), dim3(1), dim3(((p.n * 6 + 63) / 64) * 64), 0, s, p);
    return static_cast<int>(hipGetLastError());
}

template <typename real, int N>
int launch_energy_t(const EnergyParams& p, double* out, hipStream_t s) {
    hipLaunchKernelGGL((energy_kernel<real, N>), dim3(p.nblk), dim3(kThreads), 0, s, p);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, p.partial, p.nblk, out);
    return static_cast<int>(hipGetLastError());
}

}  // namespace

int launch_stage(int precision, int N, bool has_kappa, int pml_mode, const StageParams& p, hipStream_t s) {
    return precision == 0 ? launch_stage_r<double>(N, has_kappa, pml_mode, p, s)
                          : launch_stage_r<float>(N, has_kappa, pml_mode, p, s);
}

int launch_direct_apply(int precision, int N, const StageParams& p, hipStream_t s) {
    switch (N * 2 + (precision == 0 ? 0 : 1)) {
        case 2: return launch_apply<double, 1>(p, s);
        case 3: return launch_apply<float, 1>(p, s);
        case 4: return launch_apply<double, 2>(p, s);
        case 5: return launch_apply<float, 2>(p, s);
        case 6: return launch_apply<double, 3>(p, s);
        case 7: return launch_apply<float, 3>(p, s);
        case 8: return launch_apply<double, 4>(p, s);
        case 9: return launch_apply<float, 4>(p, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

int launch_probe(int precision, int N, const ProbeParams& p, hipStream_t s) {
    if (p.n <= 0) return 0;
    switch (N) {
        case 1: return precision == 0 ? launch_probe_t<double, 1>(p, s) : launch_probe_t<float, 1>(p, s);
        case 2: return precision == 0 ? launch_probe_t<double, 2>(p, s) : launch_probe_t<float, 2>(p, s);
        case 3: return precision == 0 ? launch_probe_t<double, 3>(p, s) : launch_probe_t<float, 3>(p, s);
        case 4: return precision == 0 ? launch_probe_t<double, 4>(p, s) : launch_probe_t<float, 4>(p, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

int launch_energy(int precision, int N, const EnergyParams& p, double* out, hipStream_t s) {
    switch (N) {
        case 1: return precision == 0 ? launch_energy_t<double, 1>(p, out, s) : launch_energy_t<float, 1>(p, out, s);
        case 2: return precision == 0 ? launch_energy_t<double, 2>(p, out, s) : launch_energy_t<float, 2>(p, out, s);
        case 3: return precision == 0 ? launch_energy_t<double, 3>(p, out, s) : launch_energy_t<float, 3>(p, out, s);
        case 4: return precision == 0 ? launch_energy_t<double, 4>(p, out, s) : launch_energy_t<float, 4>(p, out, s);
        default: return static_cast<int>(hipErrorInvalidValue);
    }
}

}  // namespace wdg
