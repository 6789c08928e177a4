// Matrix-core (MFMA) form of the fused stage kernel for gfx950.
//
// Same mathematics and memory layout as the scalar-operand kernel in
// kernels.hip (eqs. (26)-(29) with the upwind curl of eqs. (15)-(17), the
// weight-adjusted inverse mass of eq. (21) and the LSERK4 update), but every
// small dense product runs on the matrix cores:
//
//   Out (M x 16 elements) = Op (M x K) * X (K x 16 elements)
//
// in steps of 16 output rows and 4 columns of K.  FP32 uses one
// V_MFMA_F32_16X16X4_F32 per step.  FP64 uses up to four
// V_MFMA_F64_4X4X4_4B_F64 per step, one per 4-row group v of the 16 rows (its
// four blocks are the four 4-column groups of the 16 elements): on gfx950 that
// instruction sustains about 1.5x the FP64 rate of V_MFMA_F64_16X16X4_F64
// (76 against 49.5 TFLOP/s measured), its B operand and result lanes are those
// of register v of the 16x16x4 product, and row groups past the operator's last
// row are skipped instead of computed as padding.
//
// A tile is 16 elements (the columns), handled by six wavefronts, one per
// field component u; a workgroup takes TPW adjacent tiles (1 or 2) so that its
// wavefront count is a multiple of the four SIMDs of a compute unit.  The
// reference operators are the A operands; they are stored on the host in
// fragment order (operator tile, k-step, lane; the last tile of an N_p-row
// operator compact, see device.hpp), copied once per workgroup into LDS and
// read with one 64-lane LDS load per fragment.  Field data are the B
// operands.  The upwind flux of all six components is computed once per tile
// by its 384 threads (face node and element items) and shared through LDS, in
// one round, or in two rounds of half the face nodes each where the LDS of a
// compute unit is short.
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
//   B. R += LIFT (Fscale * upwind flux), flux read from LDS in B layout
//      (after each flux round; after A in stages with registers to spare)
//   C. R += D_r G_r + D_s G_s + D_t G_t, G_d = metric-weighted components
//   A. VF = V_q f_u, VP = V_q P_u; t1 = b VF + c VP, t2 = kappa^-1 VF - d VP
//      (eq. (9) at the cubature points); rhs_P = P_q t2 (then its LSERK
//      update); R -= P_q t1
//   D. rhs_u = P_q a^-1 V_q R (PML tiles), then the LSERK update.
#include "device.hpp"
#include <type_traits>

namespace wdg {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Out += Op X for one 16-row step: AF is the lane's A operand (FP64: the four
// words of the row groups v = 0..3), nv the number of leading row groups with
// valid rows (FP64 skips the rest; FP32 computes all 16 rows).
template <typename real>
struct Mma;
template <>
struct Mma<double> {
    using v4 = v4d;
    using AF = v4d;
    static __device__ __forceinline__ v4 run(AF a, double b, v4 c, int nv = 4) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (v < nv) c[v] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[v], b, c[v], 0, 0, 0);
        return c;
    }
};
// FP32: nv = 4 is one V_MFMA_F32_16X16X4_F32; nv < 4 marks a step whose rows all lie in the first four of
// the tile, run as one V_MFMA_F32_4X4X1_16B_F32 (a third of the cycles).  Its sixteen blocks are the
// (k, 4-column group) pairs of the step: lane 16 k + 4 c + n holds B[k][4 c + n] exactly as the 16x16x4
// product wants it, the lane's A word is row i = lane % 4 of column k, and the result register i of that
// lane accumulates row i's partial sum over the columns k of every step.  fold() adds the four partials and
// moves row g to register 0 of lane group g, the 16x16x4 result layout.
template <>
struct Mma<float> {
    using v4 = v4f;
    using AF = float;
    static __device__ __forceinline__ v4 run(AF a, float b, v4 c, int nv = 4) {
        if (nv < 4) return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ v4 fold(v4 d, int g) {
        v4 s;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float x = d[r];
            x += __shfl_xor(x, 16);
            x += __shfl_xor(x, 32);
            s[r] = x;
        }
        return v4{g == 0 ? s[0] : g == 1 ? s[1] : g == 2 ? s[2] : s[3], 0.0f, 0.0f, 0.0f};
    }
};

template <int N>
struct Ord {
    static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
    static constexpr int Nfp = (N + 1) * (N + 2) / 2;
};

// Tiles: every element block of 64 slots is four tiles of 16; PML tiles first.  A workgroup takes TPW
// adjacent tiles; its position in the launch maps to a tile group by remap_range.

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
        // uniform base + 32-bit lane offset (the rows of one tile span far less than 4 GiB)
        const unsigned lofs = static_cast<unsigned>(seg) * static_cast<unsigned>(stride_bytes) + static_cast<unsigned>(off);
        __builtin_amdgcn_global_load_lds(base + lofs, lds + c * 1024, 16, 0, 0);
    }
}

constexpr int pad1k(int bytes) { return (bytes + 1023) / 1024 * 1024; }
constexpr int kLdsCU = 160 * 1024;  // LDS of a compute unit
constexpr int wg_per_cu(int lds) { return lds <= kLdsCU ? (kLdsCU / lds < 1 ? 1 : kLdsCU / lds) : 1; }

// Per-lane global accesses as a wave-uniform base (scalar registers) plus a 32-bit lane
// offset in elements: the scalar-base addressing form, with constant node offsets folded
// into the instruction.  The offsets must stay below 4 GiB in bytes (checked on the host).
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off * static_cast<unsigned>(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, unsigned off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off * static_cast<unsigned>(sizeof(T))) = v;
}

// Compile-time shape of the kernel for one precision, order and number of
// cubature tiles.
template <typename real, int N, int QT, bool ADJ = false, int TPW = 2>
struct Shape {
    static constexpr int Np = Ord<N>::Np, Nfp = Ord<N>::Nfp, T = 16;
    static constexpr int NF = 4 * Nfp;             // face nodes per element
    static constexpr int PT = (Np + 15) / 16;      // node tiles
    static constexpr int MR = Np - 16 * (PT - 1);  // rows of the last node tile
    static constexpr int SP = (Np + 3) / 4;        // k-steps over nodes
    static constexpr int SQM = 4 * QT;             // k-steps reserved over cubature points
    static constexpr int SF = Nfp;                 // k-steps over the face nodes
    static constexpr int QMAX = 16 * QT;           // cubature points the sigma staging can hold
    static constexpr int RB = static_cast<int>(sizeof(real));
    // fragment words of each operator (V_q full tiles; P_q, D_r,s,t, LIFT compact last tile)
    static constexpr bool F64 = RB == 8;
    static constexpr int NVL = (MR + 3) / 4;       // FP64: row groups of the last node tile
    static constexpr int W_VQ = frag_words(QMAX, QT, SP, false, F64);
    static constexpr int W_PQ = frag_words(Np, PT, SQM, true, F64);
    static constexpr int W_D = frag_words(Np, PT, SP, true, F64);
    static constexpr int W_L = frag_words(Np, PT, SF, true, F64);
    static constexpr int OFF_VQ = 0, OFF_PQ = W_VQ, OFF_D = OFF_PQ + W_PQ, OFF_L = OFF_D + 3 * W_D;
    static constexpr int NW = OFF_L + W_L;
    // LDS: operator fragments (shared by the workgroup), then per tile its E,H
    // rows, sigma rows, geometry rows and neighbour offsets (all padded to whole
    // KiB for the staging copies), and per tile the flux of one round
    static constexpr int L_FR = pad1k(NW * RB);
    static constexpr int L_EH = pad1k(6 * Np * T * RB);
    static constexpr int L_SG0 = pad1k(3 * QMAX * T * RB);
    static constexpr int L_GE = pad1k(kGeo * T * RB);
    static constexpr int L_NB = pad1k(NF * T * 4);
    // The flux buffer holds the face nodes of one round: all of them (one round, two barriers
    // fewer) where that costs no workgroups per compute unit, else the first half.  Where the
    // workgroup would not fit in LDS otherwise, sigma (needed only in the PML phase) is staged into
    // the flux buffer after the flux rounds instead of with the tile.
    static constexpr int L_FL1 = 6 * NF * T * RB, L_FL2 = 6 * 4 * ((SF + 1) / 2) * T * RB;
    struct Lay {
        int lds;
        bool one, sgfl;
    };
    // LDS of the workgroup with a sigma-gradient accumulator of gl bytes per tile; force_sg
    // stages sigma into the flux buffer wherever it fits there.
    static constexpr Lay layout(int gl, bool force_sg) {
        const int nosg = L_EH + L_GE + L_NB + gl;
        const bool sg1 = (force_sg || L_FR + TPW * (nosg + L_SG0 + L_FL1) > kLdsCU) && L_FL1 >= L_SG0;
        const bool sg2 = (force_sg || L_FR + TPW * (nosg + L_SG0 + L_FL2) > kLdsCU) && L_FL2 >= L_SG0;
        const int lds1 = L_FR + TPW * (nosg + (sg1 ? 0 : L_SG0) + L_FL1);
        const int lds2 = L_FR + TPW * (nosg + (sg2 ? 0 : L_SG0) + L_FL2);
        const bool one = lds1 <= kLdsCU && wg_per_cu(lds1) == wg_per_cu(lds2);
        return Lay{one ? lds1 : lds2, one, one ? sg1 : sg2};
    }
    // Adjoint: the sigma-gradient accumulator takes LDS atomic adds from all six wavefronts.  A
    // float LDS atomic add costs about twenty times a double one on gfx950, so the accumulator is
    // double wherever that keeps the workgroups per compute unit of a float one (sigma moving
    // into the flux buffer if need be), and float otherwise.
    static constexpr Lay LAY_R = layout(ADJ ? 3 * QMAX * T * RB : 0, false);
    static constexpr Lay LAY_D0 = layout(ADJ ? 3 * QMAX * T * 8 : 0, false);
    static constexpr Lay LAY_D1 = layout(ADJ ? 3 * QMAX * T * 8 : 0, true);
    static constexpr bool keeps_wg(Lay l) { return l.lds <= kLdsCU && wg_per_cu(l.lds) >= wg_per_cu(LAY_R.lds); }
    static constexpr int barriers(Lay l) { return (l.one ? 0 : 2) + (l.sgfl ? 1 : 0); }  // beyond the least
    static constexpr bool D0_OK = keeps_wg(LAY_D0), D1_OK = keeps_wg(LAY_D1);
    static constexpr Lay LAY_D = D0_OK && (!D1_OK || barriers(LAY_D0) <= barriers(LAY_D1)) ? LAY_D0 : LAY_D1;
    static constexpr bool GL_D = ADJ && (RB == 8 || D0_OK || D1_OK);
    static constexpr Lay LAY = (!GL_D || RB == 8) ? LAY_R : LAY_D;
    static constexpr int L_GL = ADJ ? 3 * QMAX * T * (GL_D ? 8 : RB) : 0;
    static constexpr bool ONE = LAY.one;
    static constexpr int ROUNDS = ONE ? 1 : 2;
    static constexpr int S0 = ONE ? SF : (SF + 1) / 2;  // k-steps (4 face nodes each) of the first round
    static constexpr int NFH = 4 * S0;  // face nodes per flux round (the second round has NF - NFH)
    static constexpr int L_FL = ONE ? L_FL1 : L_FL2;
    static constexpr bool SGFL = LAY.sgfl;
    static constexpr int L_SG = SGFL ? 0 : L_SG0;
    static constexpr int L_TL = L_EH + L_SG + L_GE + L_NB;
    static constexpr int LDS = LAY.lds;
    // Register budget: as many wavefronts per SIMD as the workgroups that fit
    // in the 160 KiB of LDS of a compute unit bring (at most 6, 80 VGPRs).
    static constexpr int WG_PER_CU = wg_per_cu(LDS);
    static constexpr int WAVES_PER_SIMD_RAW = (WG_PER_CU * 6 * TPW + 3) / 4;
    static constexpr int WAVES_PER_SIMD = WAVES_PER_SIMD_RAW < 6 ? WAVES_PER_SIMD_RAW : 6;
};

// ADJ selects the adjoint stage (the energy-inner-product transpose of the
// stage operator; kappa = 1): q_in holds z (the weight-adjusted adjoint of the
// fields), res the stage adjoint y, q_base the running adjoint; the kernel
// writes q_base + dt L* y to q_out and adds the stage's sigma gradient to
// p.grad.  Same staging, flux, lift and curl as the forward stage, with the
// flux parameter negated by the caller.
//
// NQ > 0 fixes the number of cubature points at compile time (the stored rules of degree 2N), so that
// the guards on padded cubature slots resolve at compile time; NQ = 0 reads it from p.Nq.  RR = false is
// the form of the first Runge-Kutta stage (A_1 = 0): it reads no residual at all (the other forms read it
// when p.read_res is set).
template <typename real, int N, int QT, bool KAPPA, bool ADJ, int TPW, int NQ, int MODE = kPmlWaa, bool RR = true>
__global__ __launch_bounds__(TPW * kMfmaThreads) __attribute__((amdgpu_waves_per_eu(Shape<real, N, QT, ADJ, TPW>::WAVES_PER_SIMD)))
void stage_mfma_kernel(StageParams p) {
    static_assert(!(ADJ && KAPPA), "the adjoint stage is written for kappa = 1");
    static_assert(MODE == kPmlWaa || (!ADJ && !KAPPA), "the direct and element-constant modes are forward, kappa inside their data");
    constexpr bool WAA = MODE == kPmlWaa, DIRECT = MODE == kPmlDirect, EC = MODE == kPmlConstant;
    using M = Mma<real>;
    using v4 = typename M::v4;
    using S = Shape<real, N, QT, ADJ, TPW>;
    constexpr int QMAX = S::QMAX;
    constexpr int Np = S::Np, Nfp = S::Nfp, B = kBlock, T = S::T;
    constexpr int NF = S::NF, PT = S::PT, MR = S::MR, SP = S::SP, SQM = S::SQM, SF = S::SF, S0 = S::S0;
    constexpr bool F64 = sizeof(real) == 8;
    // flux and lift after the curl and PML terms (stages with registers to spare; not the FP32 adjoint)
    constexpr bool LATE_FLUX = (!ADJ || F64) && S::WAVES_PER_SIMD <= 4;
    // late flux of the forward weight-adjusted stage: every trace gathered (its long PML phase hides
    // them), and every per-wave row loaded from an address valid in any tile with the stage's
    // conditions applied where the value is used.  A load under a branch, or a select right after
    // it, makes the compiler wait for it there, or for every load in flight at the next use of an
    // earlier one; unconditional loads keep the wait counts exact.
    constexpr bool GATHER_ALL = LATE_FLUX && !ADJ && WAA;
    constexpr int W_D = S::W_D, OFF_VQ = S::OFF_VQ, OFF_PQ = S::OFF_PQ, OFF_D = S::OFF_D, OFF_L = S::OFF_L;
    constexpr int EHS = 6 * Np * B;
    constexpr int NFH = S::NFH;
    constexpr int FIT = (NFH * T + kMfmaThreads - 1) / kMfmaThreads;  // flux items per thread and round
    constexpr int RB = S::RB;
    constexpr int L_FR = S::L_FR, L_EH = S::L_EH, L_SG = S::L_SG, L_GE = S::L_GE, L_TL = S::L_TL;
    __shared__ __attribute__((aligned(16))) char smem[L_FR + TPW * L_TL];
    // flux [component][face node of the round][element of the tile]; sigma rows after the flux when S::SGFL
    __shared__ __attribute__((aligned(16))) real fls[TPW][6 * NFH * T];
    using GR = typename std::conditional<S::GL_D, double, real>::type;  // sigma-gradient accumulator type
    __shared__ GR gls[ADJ ? TPW * 3 * QMAX * T : 1];  // adjoint: [tile][axis][cubature point][element]

    // Workgroup: TPW adjacent tiles of one element block, six
    // wavefronts each (a multiple of four wavefronts keeps the four SIMDs of a
    // compute unit equally loaded); the operator fragments are shared.
    const int h = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kMfmaThreads);
    const int tid = static_cast<int>(threadIdx.x) - h * kMfmaThreads;
    real* fr = reinterpret_cast<real*>(smem);
    char* tl = smem + L_FR + h * L_TL;
    real* eh = reinterpret_cast<real*>(tl);
    const real* eh0 = reinterpret_cast<const real*>(smem + L_FR);  // the first tile's E,H rows
    real* sgs = S::SGFL ? fls[h] : reinterpret_cast<real*>(tl + L_EH);
    real* ges = reinterpret_cast<real*>(tl + L_EH + L_SG);
    int* nbs = reinterpret_cast<int*>(tl + L_EH + L_SG + L_GE);
    real* fl = fls[h];

    const int tile = __builtin_amdgcn_readfirstlane(
        TPW * remap_range(p.order_rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x),
                          4 / TPW * p.pml0, 4 / TPW * p.npml, 4 / TPW * p.int0, 4 / TPW * p.nint) + h);
    const int blk = tile >> 2, sub = tile & 3;
    const bool pml = blk < p.nblk_pml;
    const int Nq = NQ > 0 ? NQ : p.Nq;
    const int u = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int g = lane >> 4, j = lane & 15;
    const int e = T * sub + j;
    const real* __restrict__ qin = static_cast<const real*>(p.q_in);

    GR* gl = gls + (ADJ ? h * 3 * QMAX * T : 0);
    if constexpr (ADJ) {
        for (int i = tid; i < 3 * QMAX * T; i += kMfmaThreads) gl[i] = GR(0);
    }

    // ---- stage the tile into LDS (direct global->LDS loads)
    {
        const size_t row = static_cast<size_t>(B) * RB;  // bytes between rows of the blocked layout
        stage_rows(reinterpret_cast<const char*>(p.frags), 1024, 1024, L_FR / 1024, smem, h * 6 + u, 6 * TPW, lane);
        stage_rows(reinterpret_cast<const char*>(qin + static_cast<size_t>(blk) * EHS + T * sub), row, T * RB, 6 * Np,
                   tl, u, 6, lane);
        stage_rows(reinterpret_cast<const char*>(static_cast<const real*>(p.geo) + static_cast<size_t>(blk) * kGeo * B + T * sub),
                   row, T * RB, kGeo, tl + L_EH + L_SG, u, 6, lane);
        stage_rows(reinterpret_cast<const char*>(p.nbr + static_cast<size_t>(blk) * NF * B + T * sub), static_cast<size_t>(B) * 4,
                   T * 4, NF, tl + L_EH + L_SG + L_GE, u, 6, lane);
        if (WAA && pml && (!S::SGFL || LATE_FLUX))
            stage_rows(reinterpret_cast<const char*>(static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + T * sub),
                       row, T * RB, 3 * Nq, reinterpret_cast<char*>(sgs), u, 6, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // ---- neighbour traces for all flux rounds.  A neighbour inside one of the
    // workgroup's tiles (and the own trace at a PEC wall) is read from the staged
    // E,H rows at flux time (loc >= 0: offset from the first tile's rows) and the
    // others are gathered from global memory: here when the flux runs first, else
    // spread over the k-steps of the curl (a gather touches about one cache line
    // per lane, so a wave issuing them all at once stalls its matrix work).  With
    // GATHER_ALL every trace is gathered, the workgroup's own rows from the L2:
    // unconditional loads let the flux wait for just the loads it reads instead
    // of every load in flight.
    real nb[S::ROUNDS][FIT][6];
    int loc[S::ROUNDS][FIT], vw[S::ROUNDS][FIT], jos[S::ROUNDS][FIT];  // jos: own trace row * T + element
    {
        const int base = blk * EHS + T * (sub - h);  // the workgroup's first tile
#pragma unroll
        for (int r = 0; r < S::ROUNDS; ++r)
#pragma unroll
            for (int it = 0; it < FIT; ++it) {
                const int nitem = (r == 0 ? NFH : NF - NFH) * T;
                const int pi0 = tid + it * kMfmaThreads;
                const int pi = (pi0 < nitem ? pi0 : 0) + r * NFH * T;  // [face node][element]
                const int vv = nbs[pi];
                const int off = vv >= 0 ? vv : ~vv;
                const int rel = off - base;
                const int el = rel & (B - 1);  // element position within the workgroup's tiles
                const bool in_tile = static_cast<unsigned>(rel) < static_cast<unsigned>(Np * B) && el < TPW * T;
                vw[r][it] = vv;
                loc[r][it] = in_tile ? (el / T) * (L_TL / RB) + (rel >> 6) * T + (el & (T - 1)) : -1;
                jos[r][it] = p.fmask[r * NFH + (pi0 < nitem ? pi0 : 0) / T] * T + (pi0 & (T - 1));
                if (!LATE_FLUX && !in_tile) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) nb[r][it][c] = ldg(qin + c * Np * B, static_cast<unsigned>(off));
                }
            }
    }

    // ---- per-wave loads that only this wave needs, issued to overlap the flux phase
    // wave-uniform offsets of this tile's component-u rows (E,H part and auxiliary part); a lane
    // adds j + node * B
    const size_t ebase = static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + T * sub;
    const size_t pbase = static_cast<size_t>(p.nblk) * EHS + ebase;
    real* __restrict__ rs = static_cast<real*>(p.res);  // forward: residual; adjoint: stage adjoint y (read only)
    real* __restrict__ qo = static_cast<real*>(p.q_out);
    // base of the update (forward: q_in; adjoint: the running adjoint) and the
    // auxiliary fields entering the PML terms (forward: q_in; adjoint: y)
    const real* __restrict__ qb = ADJ ? static_cast<const real*>(p.q_base) : qin;
    const real* __restrict__ pin = ADJ ? static_cast<const real*>(p.res) : qin;
    const bool read_res = RR && p.read_res != 0;
    real bp[SP];
    real rP[PT][4], qP[PT][4], rE[PT][4];  // adjoint: qP, rE hold the update base (FP64)
#pragma unroll
    for (int s = 0; s < SP; ++s) {
        const int node = 4 * s + g;
        const int nd = ((SP * 4 == Np) || node < Np) ? node : 0;
        bp[s] = GATHER_ALL ? ldg(pin + (pml ? pbase : ebase), static_cast<unsigned>(j + nd * B))
                           : ((WAA && pml) ? ldg(pin + pbase, static_cast<unsigned>(j + nd * B)) : real(0));
    }
    // rows read only by the updates: residuals and update bases (row (kind, t, v) is item
    // (kind PT + t) 4 + v), issued a few per curl k-step (like the gathers of the late flux):
    // load_update_rows(s) issues the items of k-step s.  With GATHER_ALL a vacuum tile reads its
    // own E,H rows in place of the auxiliary rows it lacks and never uses the values.
    constexpr int NU = 3 * PT * 4;
    constexpr int UPS = (NU + SP - 1) / SP;  // update rows per curl k-step
    auto load_update_rows = [&](int s) {
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                const int nd = node < Np ? node : 0;
                const unsigned lo = static_cast<unsigned>(j + nd * B);
                if (((0 * PT + t) * 4 + v) / UPS == s)
                    rP[t][v] = GATHER_ALL ? (RR ? ldg(rs + (pml ? pbase : ebase), lo) : real(0))
                                          : ((!ADJ && !DIRECT && pml && read_res) ? ldg(rs + pbase, lo) : real(0));
                // (the adjoint reads its update base where it is used: fewer registers live through the
                // curl and the PML terms, no spills)
                if (((1 * PT + t) * 4 + v) / UPS == s)
                    qP[t][v] = GATHER_ALL ? ldg(qb + (pml ? pbase : ebase), lo)
                                          : ((!ADJ && !DIRECT && pml) ? ldg(qb + pbase, lo) : real(0));
                if (!(LATE_FLUX && !ADJ) && ((2 * PT + t) * 4 + v) / UPS == s)  // else issued before the late flux
                    rE[t][v] = ADJ ? real(0)
                                   : ((read_res && !(DIRECT && pml)) ? ldg(rs + ebase, lo) : real(0));
            }
    };
    // adjoint: this component's forward fields at the stage input, for the sigma gradient (loaded at the
    // start of the PML terms, the only place they are used, so that they are not live through the curl)
    constexpr int SPA = ADJ ? SP : 1;
    real ff[SPA], fp[SPA];

    // A operand of lane `lane` for operator tile t and k-step s (of K k-steps); the last node tile is stored
    // compact.  FP64: the four words of the row groups (layout in device.hpp); FP32: one word.
    using AF = typename M::AF;
    constexpr int NVL = S::NVL;
    const int lq = 4 * (lane & 3) + ((lane & 15) >> 2);
    const int lp = (lane >> 4) * MR + (lq < MR ? lq : MR - 1);  // FP32: lane's word in a compact tile
    // FP32 4x4x1 steps on the last node tile (at most 4 rows) and the last cubature tile (at most 4 points,
    // compile-time rule size), weight-adjusted mode: the lane's A word is row lane % 4, column lane / 16
    constexpr int QR = NQ > 0 ? NQ - 16 * (QT - 1) : 16;
    constexpr bool SMALLN = !F64 && MODE == kPmlWaa && MR <= 4;
    constexpr bool SMALLQ = !F64 && MODE == kPmlWaa && NQ > 0 && QR <= 4;
    const int ls = (lane >> 4) * MR + ((lane & 3) < MR ? (lane & 3) : MR - 1);  // ... in the compact tile
    const int lsq = (lane >> 4) * 16 + 4 * (lane & 3);                          // ... in a full V_q tile
    const int l4 = (lane >> 4) * 16 + (lane & 3) * 4;             // FP64: lane's first word in a full tile
    const int l4c = (lane >> 4) * 4 * NVL + (lane & 3) * NVL;     // FP64: ... in a compact tile
    auto frag = [&](int off, int t, int s, int K) -> AF {
        if constexpr (F64) {
            if (t < PT - 1) {
                const real* p = fr + off + (t * K + s) * 64 + l4;
                return AF{p[0], p[1], p[2], p[3]};
            }
            const real* p = fr + off + (PT - 1) * K * 64 + s * 16 * NVL + l4c;
            AF a{0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < NVL; ++v) a[v] = p[v];
            return a;
        } else {
            if (t < PT - 1) return fr[off + (t * K + s) * 64 + lane];
            return fr[off + (PT - 1) * K * 64 + s * 4 * MR + (SMALLN ? ls : lp)];
        }
    };
    auto fragq = [&](int t, int s) -> AF {
        if constexpr (F64) {
            const real* p = fr + OFF_VQ + (t * SP + s) * 64 + l4;
            return AF{p[0], p[1], p[2], p[3]};
        } else {
            return fr[OFF_VQ + (t * SP + s) * 64 + ((SMALLQ && t == QT - 1) ? lsq : lane)];
        }
    };
    // FP64: row groups with valid rows in node tile t and cubature tile t (the others are skipped); FP32: 1
    // for a 4x4x1 tile, else 4
    auto nvn = [&](int t) -> int { return F64 ? (t < PT - 1 ? 4 : NVL) : ((SMALLN && t == PT - 1) ? 1 : 4); };
    auto nvq = [&](int t) -> int {
        if constexpr (!F64) return (SMALLQ && t == QT - 1) ? 1 : 4;
        const int rows = (NQ > 0 ? NQ : QMAX) - 16 * t;
        return rows >= 16 ? 4 : (rows + 3) / 4;
    };
    // FP32 4x4x1 accumulators to the 16x16x4 layout (FP64: unchanged)
    auto fold = [&](v4 d) -> v4 {
        if constexpr (F64) return d;
        else return M::fold(d, g);
    };
    auto ehv = [&](int c, int node) -> real { return eh[(c * Np + node) * T + j]; };

    v4 R[PT];
#pragma unroll
    for (int t = 0; t < PT; ++t) R[t] = v4{0, 0, 0, 0};

    // ---- upwind flux of all six components (once per tile, shared through
    // LDS) and B. its lift for component u (eqs. (15)-(17)), in one or two rounds
    // of face nodes.  It needs the gathered neighbour traces: where registers are
    // to spare (at most four wavefronts per SIMD; FP32 adjoint excepted), it runs
    // after the curl and the PML terms, so that the gathers are in flight behind
    // that matrix work (sigma, if it lives in the flux buffer, is staged there
    // with the tile and overwritten by the flux); elsewhere it runs first.
    auto flux_and_lift = [&]() {
        const real alpha = static_cast<real>(p.alpha);
#pragma unroll
        for (int r = 0; r < S::ROUNDS; ++r) {
            const int nitem = (r == 0 ? NFH : NF - NFH) * T;
            if (r == 1) __syncthreads();  // the first round's lift has read fl
#pragma unroll
            for (int it = 0; it < FIT; ++it) {
                const int pi = tid + it * kMfmaThreads;
                if (pi >= nitem) continue;
                const int fn = r * NFH + (pi >> 4), jj = pi & 15;
                const int fc = fn / Nfp;
                const int jo = jos[r][it];
                real nv[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) nv[c] = (GATHER_ALL || loc[r][it] < 0) ? nb[r][it][c] : eh0[c * Np * T + loc[r][it]];
                const real sE = vw[r][it] >= 0 ? real(1) : real(-1);  // PEC wall: E+ = -E-, H+ = H-
                const real dEx = eh[0 * Np * T + jo] - sE * nv[0];
                const real dEy = eh[1 * Np * T + jo] - sE * nv[1];
                const real dEz = eh[2 * Np * T + jo] - sE * nv[2];
                const real dHx = eh[3 * Np * T + jo] - nv[3];
                const real dHy = eh[4 * Np * T + jo] - nv[4];
                const real dHz = eh[5 * Np * T + jo] - nv[5];
                const real nx = ges[(9 + 4 * fc) * T + jj], ny = ges[(10 + 4 * fc) * T + jj], nz = ges[(11 + 4 * fc) * T + jj];
                const real hs = real(0.5) * ges[(12 + 4 * fc) * T + jj];
                const real ndE = nx * dEx + ny * dEy + nz * dEz;
                const real ndH = nx * dHx + ny * dHy + nz * dHz;
                real* f = fl + pi;
                f[0 * NFH * T] = hs * (-(ny * dHz - nz * dHy) + alpha * (nx * ndE - dEx));
                f[1 * NFH * T] = hs * (-(nz * dHx - nx * dHz) + alpha * (ny * ndE - dEy));
                f[2 * NFH * T] = hs * (-(nx * dHy - ny * dHx) + alpha * (nz * ndE - dEz));
                f[3 * NFH * T] = hs * ((ny * dEz - nz * dEy) + alpha * (nx * ndH - dHx));
                f[4 * NFH * T] = hs * ((nz * dEx - nx * dEz) + alpha * (ny * ndH - dHy));
                f[5 * NFH * T] = hs * ((nx * dEy - ny * dEx) + alpha * (nz * ndH - dHz));
            }
            __syncthreads();
#pragma unroll
            for (int s = r * S0; s < (r == 0 ? S0 : SF); ++s) {
                const real b = fl[(u * NFH + 4 * (s - r * S0) + g) * T + j];
#pragma unroll
                for (int t = 0; t < PT; ++t) R[t] = M::run(frag(OFF_L, t, s, SF), b, R[t], nvn(t));
            }
        }
    };
    if constexpr (!LATE_FLUX) flux_and_lift();

    if constexpr (S::SGFL && !LATE_FLUX) {
        // every wave has finished reading the flux buffer: stage sigma into it (waited for before A)
        __syncthreads();
        if (WAA && pml)
            stage_rows(reinterpret_cast<const char*>(static_cast<const real*>(p.sigma) + static_cast<size_t>(blk) * 3 * Nq * B + T * sub),
                       static_cast<size_t>(B) * RB, T * RB, 3 * Nq, reinterpret_cast<char*>(fl), u, 6, lane);
    }

    const int SQ = (Nq + 3) / 4;
    const int ax = (u < 3) ? u : u - 3;
    const int bb = (ax == 2) ? 0 : ax + 1;
    const int cc = (ax == 0) ? 2 : ax - 1;
    const real rkA = static_cast<real>(p.rk_a), rkB = static_cast<real>(p.rk_b);
    // adjoint: y_next = yn_a (y_scale y) + yn_b q_hat_out, y being this stage's input
    real* __restrict__ yn = ADJ ? static_cast<real*>(p.y_next) : nullptr;
    const real yna = static_cast<real>(p.yn_a * p.y_scale), ynb = static_cast<real>(p.yn_b);
    // time step of this lane's element (a per-element scale lets independent simulations share a launch)
    const real dt = static_cast<real>(p.dt_scale ? p.dt * p.dt_scale[static_cast<size_t>(blk) * B + e] : p.dt);

    // ---- C. volume curl: +curl H (E components), -curl E (H components)
    {
        const int fo = (u < 3) ? 3 : 0;
        const real sgn = (u < 3) ? real(1) : real(-1);
        const real rb = sgn * ges[bb * T + j], rc = sgn * ges[cc * T + j];
        const real sb = sgn * ges[(3 + bb) * T + j], sc = sgn * ges[(3 + cc) * T + j];
        const real tb = sgn * ges[(6 + bb) * T + j], tc = sgn * ges[(6 + cc) * T + j];
        constexpr int NG = S::ROUNDS * FIT * 6, GPS = (NG + SP - 1) / SP;  // gathers, per k-step
#pragma unroll
        for (int s = 0; s < SP; ++s) {
            load_update_rows(s);
            if constexpr (LATE_FLUX) {
#pragma unroll
                for (int ig = s * GPS; ig < (s + 1) * GPS && ig < NG; ++ig) {
                    const int c = ig % 6, it = (ig / 6) % FIT, r = ig / (6 * FIT);
                    if (GATHER_ALL || loc[r][it] < 0) {
                        const int vv = vw[r][it], off = vv >= 0 ? vv : ~vv;
                        nb[r][it][c] = ldg(qin + c * Np * B, static_cast<unsigned>(off));
                    }
                }
            }
            const int node = 4 * s + g;
            const bool ok = (SP * 4 == Np) || node < Np;
            const real xb = ok ? ehv(fo + bb, node) : real(0);
            const real xc = ok ? ehv(fo + cc, node) : real(0);
            const real gr = rb * xc - rc * xb, gs = sb * xc - sc * xb, gt = tb * xc - tc * xb;
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                R[t] = M::run(frag(OFF_D + 0 * W_D, t, s, SP), gr, R[t], nvn(t));
                R[t] = M::run(frag(OFF_D + 1 * W_D, t, s, SP), gs, R[t], nvn(t));
                R[t] = M::run(frag(OFF_D + 2 * W_D, t, s, SP), gt, R[t], nvn(t));
            }
        }
    }

    if constexpr (S::SGFL && !LATE_FLUX) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    // LSERK update of the auxiliary component from its right-hand side RP
    auto aux_update = [&](const v4* RP) {
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                if (node < Np) {
                    const unsigned lo = static_cast<unsigned>(j + node * B);
                    if constexpr (ADJ) {
                        const real qn = ldg(qb + pbase, lo) + dt * RP[t][v];
                        stg(qo + pbase, lo, qn);
                        if (yn) stg(yn + pbase, lo, yna * ldg(rs + pbase, lo) + ynb * qn);  // rs holds y here
                    } else {
                        const real r = dt * RP[t][v] + rkA * ((GATHER_ALL && !read_res) ? real(0) : rP[t][v]);
                        stg(rs + pbase, lo, r);
                        stg(qo + pbase, lo, qP[t][v] + rkB * r);
                    }
                }
            }
    };

    // ---- A. PML terms at the cubature points (eqs. (26)-(29))
    if (WAA && pml) {
        const real* __restrict__ kp =
            KAPPA ? static_cast<const real*>(p.kappa) + static_cast<size_t>(blk) * 3 * Nq * B + e : nullptr;
        // One cubature tile (16 points) at a time, so that only its products are live:
        // forward: VF = V_q f_u, VP = V_q P_u; adjoint: VF = V_q z_u, VP = V_q y_{P,u} and, for
        // the gradient, VFf = V_q f_u, VPf = V_q P_u of the forward stage input.  Then eq. (9) at
        // cubature point q = 16 tq + 4 v + g.  Forward: VF <- -t1, VP <- t2.  Adjoint: VF <- b VZ -
        // kappa^-1 VY, VP <- -c VZ - d VY, and the node's sigma gradient (kappa = 1: db/dsigma_(u,v,w)
        // = (-1, 1, 1), dc/dsigma_(u,v,w) = (sigma_u - b, sigma_w - sigma_u, sigma_v - sigma_u),
        // dd/dsigma_u = 1) goes to the LDS accumulator, weighted by dt J w_q.  Last rhs_P += P_q t2 and
        // R -= P_q t1 over the tile's k-steps.
        const double wJ = ADJ ? p.dt * p.Jk[static_cast<size_t>(blk) * B + e] : 0.0;
        if constexpr (ADJ) {
            const real* __restrict__ qf = static_cast<const real*>(p.q_fwd);
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                const int node = 4 * s + g;
                const int nd = ((SP * 4 == Np) || node < Np) ? node : 0;
                ff[s] = ldg(qf + ebase, static_cast<unsigned>(j + nd * B));
                fp[s] = ldg(qf + pbase, static_cast<unsigned>(j + nd * B));
            }
        }
        v4 RP[PT];
#pragma unroll
        for (int t = 0; t < PT; ++t) RP[t] = v4{0, 0, 0, 0};
#pragma unroll
        for (int tq = 0; tq < QT; ++tq) {
            v4 VF = v4{0, 0, 0, 0}, VP = v4{0, 0, 0, 0}, VFf = v4{0, 0, 0, 0}, VPf = v4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < SP; ++s) {
                const int node = 4 * s + g;
                const bool ok = (SP * 4 == Np) || node < Np;
                const AF a = fragq(tq, s);
                VF = M::run(a, ok ? ehv(u, node) : real(0), VF, nvq(tq));
                VP = M::run(a, ok ? bp[s] : real(0), VP, nvq(tq));
                if constexpr (ADJ) {
                    VFf = M::run(a, ok ? ff[s] : real(0), VFf, nvq(tq));
                    VPf = M::run(a, ok ? fp[s] : real(0), VPf, nvq(tq));
                }
            }
            if (SMALLQ && tq == QT - 1) {
                VF = fold(VF);
                VP = fold(VP);
                if constexpr (ADJ) {
                    VFf = fold(VFf);
                    VPf = fold(VPf);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 16 * tq + 4 * v + g;
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
                    const real vf = VF[v], vp = VP[v];
                    if constexpr (ADJ) {
                        const real vff = VFf[v], vpf = VPf[v];
                        const real w = static_cast<real>(wJ * p.cub_w[q]);
                        const real gu = -vf * (-vff + (sa - bq) * vpf) - vp * vpf;
                        const real gv = -vf * (vff + (scq - sa) * vpf);
                        const real gw = -vf * (vff + (sbq - sa) * vpf);
                        atomicAdd(&gl[(ax * QMAX + q) * T + j], static_cast<GR>(w * gu));
                        atomicAdd(&gl[(bb * QMAX + q) * T + j], static_cast<GR>(w * gv));
                        atomicAdd(&gl[(cc * QMAX + q) * T + j], static_cast<GR>(w * gw));
                        t1 = kinv * vp - bq * vf;
                        t2 = -cq * vf - dq * vp;
                    } else {
                        t1 = bq * vf + cq * vp;
                        t2 = kinv * vf - dq * vp;
                    }
                }
                VF[v] = -t1;
                VP[v] = t2;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int sq = 4 * tq + v;
                if (sq < SQ) {
#pragma unroll
                    for (int t = 0; t < PT; ++t) {
                        const AF a = frag(OFF_PQ, t, sq, SQM);
                        RP[t] = M::run(a, VP[v], RP[t], nvn(t));
                        R[t] = M::run(a, VF[v], R[t], nvn(t));
                    }
                }
            }
        }
        if constexpr (SMALLN) RP[PT - 1] = fold(RP[PT - 1]);
        aux_update(RP);
    }

    // ---- A'. element-constant scheme: eq. (9) pointwise at the nodes with the element's sigma,
    // kappa (sampled at its node farthest beyond the interface); rhs = a^-1 (R - b f - c P)
    real ainv = real(1);
    if (EC && pml) {
        const real* __restrict__ ec = static_cast<const real*>(p.pml_mats) + static_cast<size_t>(blk) * 6 * B + e;
        const real sa = ec[ax * B], sbe = ec[bb * B], sce = ec[cc * B];
        const real ka = ec[(3 + ax) * B], kb = ec[(3 + bb) * B], kc = ec[(3 + cc) * B];
        const real kinv = real(1) / ka;
        const real a = kb * kc * kinv;
        const real bq = (sbe * kc + sce * kb - a * sa) * kinv;
        const real cq = sbe * sce - bq * sa;
        const real dq = sa * kinv;
        ainv = ka / (kb * kc);
        v4 RP[PT];
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                const real f = node < Np ? ehv(u, node) : real(0), P = qP[t][v];
                R[t][v] -= bq * f + cq * P;
                RP[t][v] = kinv * f - dq * P;
            }
        aux_update(RP);
    }

    if constexpr (LATE_FLUX) {
        if constexpr (!ADJ) {  // the residual rows of the final update, in flight behind the flux
#pragma unroll
            for (int t = 0; t < PT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int node = 16 * t + 4 * v + g;
                    const int nd = node < Np ? node : 0;
                    rE[t][v] = GATHER_ALL ? (RR ? ldg(rs + ebase, static_cast<unsigned>(j + nd * B)) : real(0))
                                          : ((read_res && !(DIRECT && pml)) ? ldg(rs + ebase, static_cast<unsigned>(j + nd * B)) : real(0));
                }
        }
        if constexpr (S::SGFL) __syncthreads();  // every wave has read sigma from the flux buffer
        flux_and_lift();
    }

    // every product into R is done: its 4x4x1 tile to the 16x16x4 layout
    if constexpr (SMALLN) R[PT - 1] = fold(R[PT - 1]);

    // ---- dipole source on the electric components (not part of the adjoint operator)
    if (!ADJ && u < 3) {
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

    // ---- direct scheme: the PML tile's vacuum right-hand side goes to the work buffer; its PML
    // terms and update follow in the apply kernel
    if (DIRECT && pml) {
        real* __restrict__ wo = static_cast<real*>(p.pml_work) + static_cast<size_t>(blk) * EHS + static_cast<size_t>(u) * Np * B + e;
#pragma unroll
        for (int t = 0; t < PT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int node = 16 * t + 4 * v + g;
                if (node < Np) wo[node * B] = R[t][v];
            }
        return;
    }
    if (EC && pml) {
#pragma unroll
        for (int t = 0; t < PT; ++t) R[t] *= ainv;
    }

    // ---- D. weight-adjusted inverse mass on PML tiles: rhs = P_q a^-1 V_q R (eq. (21));
    // in the adjoint it acts before the curl (on y, giving z).  Applied on every PML tile
    // unless the caller opted out where it is the identity (kappa = 1, rule exact to degree 2N).
    if (!ADJ && WAA && pml && (KAPPA || !p.waa_skip)) {
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
                    for (int t = 0; t < QT; ++t) Z[t] = M::run(fragq(t, sp), R[tp][v], Z[t], nvq(t));
                }
            }
        if constexpr (SMALLQ) Z[QT - 1] = fold(Z[QT - 1]);
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
                    for (int t = 0; t < PT; ++t) O[t] = M::run(frag(OFF_PQ, t, sq, SQM), Z[tq][v], O[t], nvn(t));
                }
            }
        if constexpr (SMALLN) O[PT - 1] = fold(O[PT - 1]);
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
                const unsigned lo = static_cast<unsigned>(j + node * B);
                if constexpr (ADJ) {
                    // L* y = -L_vac(-alpha) z + P_q(-b VZ + kappa^-1 VY) = -R
                    const real qn = ldg(qb + ebase, lo) - dt * R[t][v];
                    stg(qo + ebase, lo, qn);
                    if (yn) stg(yn + ebase, lo, yna * ehv(u, node) + ynb * qn);
                } else {
                    const real r = dt * R[t][v] + rkA * ((GATHER_ALL && !read_res) ? real(0) : rE[t][v]);
                    stg(rs + ebase, lo, r);
                    stg(qo + ebase, lo, ehv(u, node) + rkB * r);
                }
            }
        }

    // ---- adjoint: add the tile's sigma gradient (all six components summed) to p.grad
    if constexpr (ADJ) {
        if (pml) {
            __syncthreads();
            double* __restrict__ gd = p.grad + static_cast<size_t>(blk) * 3 * Nq * B + T * sub;
            for (int i = tid; i < 3 * Nq * T; i += kMfmaThreads) {
                const int jj = i & (T - 1), aq = i >> 4;  // aq = axis * Nq + q
                const int a = aq / Nq, q = aq - a * Nq;
                gd[static_cast<size_t>(aq) * B + jj] += static_cast<double>(gl[(a * QMAX + q) * T + jj]);
            }
        }
    }
}

// Points of the stored cubature rules of degree 2N.
template <int N>
constexpr int rule_nq() { return N == 1 ? 4 : N == 2 ? 14 : N == 3 ? 24 : 51; }

template <typename real, int N, int QT, bool K, bool ADJ, int TPW, int MODE = kPmlWaa>
int launch_t(const StageParams& p, hipStream_t s) {
    if constexpr (Shape<real, N, QT, ADJ, TPW>::LDS > 160 * 1024) {
        return static_cast<int>(hipErrorInvalidConfiguration);  // more LDS than a compute unit has
    } else {
        if (p.npml + p.nint == 0) return 0;
        const dim3 grid(4 / TPW * (p.npml + p.nint)), block(TPW * kMfmaThreads);
        constexpr int RQ = rule_nq<N>();
        if constexpr (MODE == kPmlWaa && !K && (RQ + 15) / 16 == QT) {
            if (p.Nq == RQ) {
                bool first = false;  // the first Runge-Kutta stage of the forward scheme: no residual loads
                if constexpr (!ADJ) first = !p.read_res;
                if constexpr (!ADJ) {
                    if (first) hipLaunchKernelGGL((stage_mfma_kernel<real, N, QT, K, ADJ, TPW, RQ, kPmlWaa, false>), grid, block, 0, s, p);
                }
                if (!first) hipLaunchKernelGGL((stage_mfma_kernel<real, N, QT, K, ADJ, TPW, RQ>), grid, block, 0, s, p);
                return static_cast<int>(hipGetLastError());
            }
        }
        hipLaunchKernelGGL((stage_mfma_kernel<real, N, QT, K, ADJ, TPW, 0, MODE>), grid, block, 0, s, p);
        return static_cast<int>(hipGetLastError());
    }
}

template <typename real, int N, int QT>
constexpr bool adj_fits() { return Shape<real, N, QT, true, 2>::LDS <= 160 * 1024; }

template <typename real, int N, int QT>
int launch_k(bool k, int tpw, int mode, const StageParams& p, hipStream_t s) {
    if (mode == kPmlDirect)
        return tpw == 1 ? launch_t<real, N, QT, false, false, 1, kPmlDirect>(p, s) : launch_t<real, N, QT, false, false, 2, kPmlDirect>(p, s);
    if (mode == kPmlConstant)
        return tpw == 1 ? launch_t<real, N, QT, false, false, 1, kPmlConstant>(p, s)
                        : launch_t<real, N, QT, false, false, 2, kPmlConstant>(p, s);
    if (tpw == 1) return k ? launch_t<real, N, QT, true, false, 1>(p, s) : launch_t<real, N, QT, false, false, 1>(p, s);
    return k ? launch_t<real, N, QT, true, false, 2>(p, s) : launch_t<real, N, QT, false, false, 2>(p, s);
}

template <typename real>
int launch_adj(int N, int QT, const StageParams& p, hipStream_t s) {
    switch (N * 10 + QT) {
        case 11: return launch_t<real, 1, 1, false, true, 2>(p, s);
        case 12: return launch_t<real, 1, 2, false, true, 2>(p, s);
        case 21: return launch_t<real, 2, 1, false, true, 2>(p, s);
        case 22: return launch_t<real, 2, 2, false, true, 2>(p, s);
        case 32: return launch_t<real, 3, 2, false, true, 2>(p, s);
        case 33: return launch_t<real, 3, 3, false, true, 2>(p, s);
        default: return -1;
    }
}

// Order / cubature-tile combinations with a matrix-core kernel.  FP64 at
// N = 4 would need more than the 160 KiB of LDS of a compute unit.
template <typename real>
int launch_r(int N, int QT, bool k, int tpw, int mode, const StageParams& p, hipStream_t s) {
    switch (N * 10 + QT) {
        case 11: return launch_k<real, 1, 1>(k, tpw, mode, p, s);
        case 12: return launch_k<real, 1, 2>(k, tpw, mode, p, s);
        case 21: return launch_k<real, 2, 1>(k, tpw, mode, p, s);
        case 22: return launch_k<real, 2, 2>(k, tpw, mode, p, s);
        case 32: return launch_k<real, 3, 2>(k, tpw, mode, p, s);
        case 33: return launch_k<real, 3, 3>(k, tpw, mode, p, s);
        default: return -1;
    }
}

template <typename real>
int launch_r4(int QT, bool k, int tpw, int mode, const StageParams& p, hipStream_t s) {
    switch (QT) {
        case 3: return launch_k<real, 4, 3>(k, tpw, mode, p, s);
        case 4: return launch_k<real, 4, 4>(k, tpw, mode, p, s);
        default: return -1;
    }
}

template <typename real, int N, int QT>
constexpr bool fits(int tpw) {
    return tpw == 1 ? Shape<real, N, QT, false, 1>::LDS <= 160 * 1024 : Shape<real, N, QT, false, 2>::LDS <= 160 * 1024;
}

}  // namespace

bool adjoint_supported(int N, int Nq, int precision) {
    if (!mfma_supported(N, Nq, precision)) return false;
    const int QT = (Nq + 15) / 16;
    const bool f64 = precision == 0;
    switch (N * 10 + QT) {
        case 11: return f64 ? adj_fits<double, 1, 1>() : adj_fits<float, 1, 1>();
        case 12: return f64 ? adj_fits<double, 1, 2>() : adj_fits<float, 1, 2>();
        case 21: return f64 ? adj_fits<double, 2, 1>() : adj_fits<float, 2, 1>();
        case 22: return f64 ? adj_fits<double, 2, 2>() : adj_fits<float, 2, 2>();
        case 32: return f64 ? adj_fits<double, 3, 2>() : adj_fits<float, 3, 2>();
        case 33: return f64 ? adj_fits<double, 3, 3>() : adj_fits<float, 3, 3>();
        case 43: return !f64 && adj_fits<float, 4, 3>();
        case 44: return !f64 && adj_fits<float, 4, 4>();
        default: return false;
    }
}

bool mfma_supported(int N, int Nq, int precision) {
    const int QT = (Nq + 15) / 16;
    switch (N * 10 + QT) {
        case 11: case 12: case 21: case 22: case 32: case 33: case 43: case 44: return true;
        default: return false;
    }
}

bool mfma_tiles_fit(int N, int Nq, int precision, int tpw) {
    if (!mfma_supported(N, Nq, precision)) return false;
    const int QT = (Nq + 15) / 16;
    const bool d = precision == 0;
    switch (N * 10 + QT) {
        case 11: return d ? fits<double, 1, 1>(tpw) : fits<float, 1, 1>(tpw);
        case 12: return d ? fits<double, 1, 2>(tpw) : fits<float, 1, 2>(tpw);
        case 21: return d ? fits<double, 2, 1>(tpw) : fits<float, 2, 1>(tpw);
        case 22: return d ? fits<double, 2, 2>(tpw) : fits<float, 2, 2>(tpw);
        case 32: return d ? fits<double, 3, 2>(tpw) : fits<float, 3, 2>(tpw);
        case 33: return d ? fits<double, 3, 3>(tpw) : fits<float, 3, 3>(tpw);
        case 43: return d ? fits<double, 4, 3>(tpw) : fits<float, 4, 3>(tpw);
        case 44: return d ? fits<double, 4, 4>(tpw) : fits<float, 4, 4>(tpw);
        default: return false;
    }
}

int launch_adjoint_mfma(int precision, int N, const StageParams& p, hipStream_t s) {
    const int QT = (p.Nq + 15) / 16;
    if (N == 4) return precision == 0 ? -1 : (QT == 3 ? launch_t<float, 4, 3, false, true, 2>(p, s)
                                                      : QT == 4 ? launch_t<float, 4, 4, false, true, 2>(p, s) : -1);
    return precision == 0 ? launch_adj<double>(N, QT, p, s) : launch_adj<float>(N, QT, p, s);
}

int launch_stage_mfma(int precision, int N, bool has_kappa, int tpw, int pml_mode, const StageParams& p, hipStream_t s) {
    const int QT = (p.Nq + 15) / 16;
    int e;
    if (N == 4)
        e = precision == 0 ? launch_r4<double>(QT, has_kappa, tpw, pml_mode, p, s) : launch_r4<float>(QT, has_kappa, tpw, pml_mode, p, s);
    else
        e = precision == 0 ? launch_r<double>(N, QT, has_kappa, tpw, pml_mode, p, s) : launch_r<float>(N, QT, has_kappa, tpw, pml_mode, p, s);
    // the direct scheme's PML terms and update of the PML blocks
    if (e == 0 && pml_mode == kPmlDirect) e = launch_direct_apply(precision, N, p, s);
    return e;
}

}  // namespace wdg
