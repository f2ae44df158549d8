// psm_kernels.hip -- gfx950 kernels of the PSM-LBM hot path.
//
// Method: Kemmler et al., arXiv 2303.11811.
//   Sec. 2.1   D3Q19 SRT collision with forcing, eqs. (1)-(8)
//   Sec. 2.3   PSM collision, solid operator, particle velocity at the cell
//              centre, hydrodynamic force and torque, eqs. (17)-(22)
//   Sec. 2.3.2 linear-approximation solid fraction, eqs. (25)-(27)
//   Sec. 3.1   GPU time step: mapping -> PSM kernel -> force reduction
//
// Storage is pull-scheme: grid[p] holds the post-collision PDFs of the last
// step at their source cell, so a cell gathers f_q(x,t) = grid[p][q][x - c_q]
// (eq. 2 read backwards), collides, and writes grid[p^1][q][x] aligned.
// The paper's separate mapping / setU / redF kernels are fused into the
// stream-collide launch: each workgroup stages its tile's sphere candidates in
// LDS, maps solid fractions in registers, evaluates U_p(x) (eq. 20) on the fly
// and sums the per-sphere force/torque of its tile deterministically.
#include "psm_internal.h"

#include <mutex>

namespace psm {

// ---------------------------------------------------------------------------
// PDF access of the step kernel through buffer resources. A resource covers
// one z-plane of a grid (raw bytes, fewer than 2^31); every load or store
// takes the cell's byte offset inside the plane per lane and the run of its
// direction (q * 64 values) as a scalar offset, so that no per-access 64-bit
// address arithmetic runs on the vector ALU.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
constexpr int RSRC_WORD3 = 0x00020000;   // raw 32-bit data format, no swizzle

// Cache policy of the PDF streams (compile-time switches, measured by the
// tuning sweeps): nontemporal stores / loads bypass cache retention.
#ifndef PSM_NT_STORE
#define PSM_NT_STORE 1
#endif
#ifndef PSM_NT_LOAD
#define PSM_NT_LOAD 0
#endif
constexpr int LD_AUX = PSM_NT_LOAD ? 2 : 0;
constexpr int ST_AUX = PSM_NT_STORE ? 2 : 0;

#ifndef PSM_BUFFER_IO
#define PSM_BUFFER_IO 1
#endif
#if PSM_BUFFER_IO
__device__ __forceinline__ Rsrc plane_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, RSRC_WORD3);
}
#define PSM_LD(B, T, r, vo, so) __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_##B(r, vo, so, LD_AUX))
#define PSM_ST(B, U, v, r, vo, so) __builtin_amdgcn_raw_buffer_store_##B(__builtin_bit_cast(U, v), r, vo, so, ST_AUX)
#else
// plain global accesses from the plane's base address (compile-time alternative)
typedef const char* RsrcPtr;
#define Rsrc RsrcPtr
__device__ __forceinline__ Rsrc plane_rsrc(const void* base, unsigned) { return (const char*)base; }
#define GLB __attribute__((address_space(1)))
#define PSM_LD(B, T, r, vo, so) (*(const GLB T*)((r) + (so) + (vo)))
#define PSM_ST(B, U, v, r, vo, so) __builtin_nontemporal_store(v, (GLB decltype(v)*)((r) + (so) + (vo)))
#endif

// ---------------------------------------------------------------------------
// Storage traits: FP64 stores f; the deviation forms store d = f - w_q
// (FP16 as scale * d) and compute in FP32.
struct St64 {
    using T = double;
    using R = double;
    static constexpr bool DEV = false;
    static constexpr bool SCALED = false;
    __device__ static R ld(Rsrc r, unsigned vo, int so) { return PSM_LD(b64, double, r, vo, so); }
    __device__ static void st(Rsrc r, unsigned vo, int so, R v) { PSM_ST(b64, u32x2, v, r, vo, so); }
    __device__ static double to_f64(T v, float) { return v; }
    __device__ static T from_f64(double v, float) { return v; }
};
struct St32 {
    using T = float;
    using R = float;
    static constexpr bool DEV = true;
    static constexpr bool SCALED = false;
    __device__ static R ld(Rsrc r, unsigned vo, int so) { return PSM_LD(b32, float, r, vo, so); }
    __device__ static void st(Rsrc r, unsigned vo, int so, R v) { PSM_ST(b32, unsigned int, v, r, vo, so); }
    __device__ static double to_f64(T v, float) { return (double)v; }
    __device__ static T from_f64(double v, float) { return (float)v; }
};
struct St16 {
    using T = _Float16;
    using R = float;
    static constexpr bool DEV = true;
    // The step kernel works on the stored scaled deviations s d directly (the
    // scale s is folded into the collision constants), so its loads and
    // stores are bare conversions. State I/O converts with the scale.
    static constexpr bool SCALED = true;
    __device__ static R ld(Rsrc r, unsigned vo, int so) { return (float)PSM_LD(b16, _Float16, r, vo, so); }
    __device__ static void st(Rsrc r, unsigned vo, int so, R v) {
        const _Float16 h = (_Float16)v;
        PSM_ST(b16, unsigned short, h, r, vo, so);
    }
    // scale is a power of two: multiplication by it and by 1/scale is exact
    __device__ static double to_f64(T v, float inv) { return (double)((float)v * inv); }
    __device__ static T from_f64(double v, float scale) { return (_Float16)(float)(v * (double)scale); }
};

// The box constant of the collision's precision R: the FP64 value or its
// FP32 copy (both set by the host).
template <class R> __device__ __forceinline__ R pick(double d, float f);
template <> __device__ __forceinline__ double pick<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float pick<float>(double, float f) { return f; }

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline int find_box(const int* tile_base, int nbox, int t) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (tile_base[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Cross-lane moves on the vector ALU. DPP forms stay inside a row of 16
// lanes: quad permutations, the mirror inside each half row (lane i <-> 7 - i
// of its group of 8) and the rotation of a row by 8 (lane i <-> i ^ 8).
// Across rows, the gfx950 swaps exchange odd with even rows (lanes i and
// i ^ 16) and the two halves of the wave (lanes i and i ^ 32): with both
// operands the same value v, the two results are v at the lower partner and
// v at the upper partner, so their sum is the pair sum, taken in the same
// order on both lanes.
template <int CTRL> __device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_ROR8 = 0x128;

__device__ __forceinline__ float pair_sum16(float v) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float pair_sum32(float v) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double join(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double pair_sum16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return join(l[0], h[0]) + join(l[1], h[1]);
}
__device__ __forceinline__ double pair_sum32(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    return join(l[0], h[0]) + join(l[1], h[1]);
}
template <int CTRL> __device__ __forceinline__ float dppv(float v) { return dpp_f32<CTRL>(v); }
template <int CTRL> __device__ __forceinline__ double dppv(double v) { return dpp_f64<CTRL>(v); }

// Wave sums of six values at once (V = float or double). Inside each group
// of 8 lanes a butterfly splits the values (padded to 8) between exchanging
// lanes: the mirror pair by bit 2 of the lane, then quad partners by bits 1
// and 0 (7 exchanges), after which lane l holds the group's sum of value
// l & 7; three exchanges across groups (row rotation by 8, the row swap, the
// half swap) finish the sums. Lane l returns the total of value l & 7
// (values 6 and 7 are padding). The order of the additions is fixed, so the
// result is reproducible bit for bit.
template <class V>
__device__ inline V wave_sum6(const V v[6], int lane) {
    const bool b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
    V a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const V lo = v[i], hi = i + 4 < 6 ? v[i + 4] : (V)0;
        const V keep = b2 ? hi : lo, send = b2 ? lo : hi;
        a[i] = keep + dppv<DPP_ROW_HALF_MIRROR>(send);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const V keep = b1 ? a[i + 2] : a[i], send = b1 ? a[i] : a[i + 2];
        b[i] = keep + dppv<DPP_QUAD_XOR2>(send);
    }
    const V keep = b0 ? b[1] : b[0], send = b0 ? b[0] : b[1];
    V d = keep + dppv<DPP_QUAD_XOR1>(send);
    d += dppv<DPP_ROW_ROR8>(d);
    d = pair_sum16(d);
    return pair_sum32(d);
}

// Uniform (wave-invariant) data is read through the constant address space so
// that it lands in scalar registers.
#define PSM_CONST __attribute__((address_space(4)))
template <class T> __device__ __forceinline__ const PSM_CONST T* cptr(const T* p) {
    return (const PSM_CONST T*)p;
}

// ---------------------------------------------------------------------------
// Lattice products of direction Q with only its nonzero terms (D3Q19
// components are 0 or +-1; at most two are nonzero), in x, y, z order.
template <int C, class R> __device__ __forceinline__ R cterm(R v) { return C > 0 ? v : -v; }
template <class R, int Q> __device__ __forceinline__ R cdot(R x, R y, R z) {
    constexpr int a = CX[Q], b = CY[Q], c = CZ[Q];
    if constexpr (a != 0 && b != 0) return cterm<a>(x) + cterm<b>(y);
    else if constexpr (a != 0 && c != 0) return cterm<a>(x) + cterm<c>(z);
    else if constexpr (b != 0 && c != 0) return cterm<b>(y) + cterm<c>(z);
    else if constexpr (a != 0) return cterm<a>(x);
    else if constexpr (b != 0) return cterm<b>(y);
    else if constexpr (c != 0) return cterm<c>(z);
    else return (R)0;
}
// c.M.c for a symmetric M given as the diagonal (Mxx, Myy, Mzz) and the
// doubled off-diagonal terms (2 Mxy, 2 Mxz, 2 Myz).
template <class R, int Q>
__device__ __forceinline__ R cmc(R Mxx, R Myy, R Mzz, R Mxy2, R Mxz2, R Myz2) {
    constexpr int a = CX[Q], b = CY[Q], c = CZ[Q];
    if constexpr (a != 0 && b != 0) return (a * b > 0) ? (Mxx + Myy) + Mxy2 : (Mxx + Myy) - Mxy2;
    else if constexpr (a != 0 && c != 0) return (a * c > 0) ? (Mxx + Mzz) + Mxz2 : (Mxx + Mzz) - Mxz2;
    else if constexpr (b != 0 && c != 0) return (b * c > 0) ? (Myy + Mzz) + Myz2 : (Myy + Mzz) - Myz2;
    else if constexpr (a != 0) return Mxx;
    else if constexpr (b != 0) return Myy;
    else return Mzz;
}

// Per weight class W (axis or diagonal) of a cell: the terms of the SRT
// update with forcing (eqs. 3, 5, 8) that do not depend on the direction.
//   E_q(U) = W (base + k45 (c.U)^2) + 3 W (c.U) = s + a,  E_qbar(U) = s - a,
//   F_q = fa + fs (c.U) - pu,  F_qbar = -fa + fs (c.U) - pu,  base = rho - k15 U.U
template <class R>
struct WClass {
    R Wb;      // W base (per cell)
    R owb_pu;  // omega W base - pu (per cell)
    R Wk;      // W k45 (box constant)
    R W3;      // 3 W
    R owk;     // omega W k45 (box constant)
    R ow3;     // 3 omega W (box constant)
};

// One inverse pair (q, q+1) of the plain update f~ = f + omega (E - f) + F:
//   f~_q = (1 - omega) f_q + P + A,  f~_qbar = (1 - omega) f_qbar + P - A,
//   P = omega s + fs (c.U) - pu,  A = omega a + fa.
template <class R, int Q>
__device__ __forceinline__ void pair_fluid(R& fq, R& fb, R cu, const WClass<R>& w, R fa, R fs, R om1) {
    const R P = fmar(fs, cu, fmar(w.owk, cu * cu, w.owb_pu));
    const R A = fmar(w.ow3, cu, fa);
    fq = fmar(om1, fq, P + A);
    fb = fmar(om1, fb, P - A);
}

// The same pair under PSM (eqs. 17-19):
//   f~_q = f_q + (1-B) t_q + B (f_qbar - E_qbar(U) - f_q) + sum_s B_s E_q(V_s),
//   t_q = omega (E_q(U) - f_q) + F_q,
// with the slot sum folded into ten cell scalars:
//   sum_s B_s E_q(V_s) = W (A0 + k45 c.M.c) + 3 W c.P,
//   A0 = sum_s B_s (rho - k15 V_s.V_s), M = sum_s B_s V_s V_s^T, P = sum_s B_s V_s.
// Collected by parity in c_q, with alpha = 1 - (1-B) omega - B, beta = (1-B) omega - B
// and gamma = (1-B) omega + B (per cell):
//   f~_q    = alpha f_q + B f_qbar + Sym + Anti,  f~_qbar = alpha f_qbar + B f_q + Sym - Anti,
//   Sym  = [beta W base - (1-B) pu + W A0] + beta W k45 (c.U)^2 + (1-B) fs (c.U) + W k45 c.M.c,
//   Anti = gamma 3 W (c.U) + (1-B) fa + 3 W c.P,
// where the bracket (C1), beta W k45 (C2) and gamma 3 W (C3) are per weight class.
template <class R, int Q>
__device__ __forceinline__ void pair_psm(R& fq, R& fb, R cu, R C1, R C2, R C3, R Wk, R W3, R ofs, R ofa, R alpha,
                                         R Bt, R cM, R cP) {
    const R Sym = fmar(C2, cu * cu, fmar(ofs, cu, fmar(Wk, cM, C1)));
    const R Anti = fmar(C3, cu, fmar(W3, cP, ofa));
    const R nq = fmar(alpha, fq, fmar(Bt, fb, Sym + Anti));
    const R nb = fmar(alpha, fb, fmar(Bt, fq, Sym - Anti));
    fq = nq;
    fb = nb;
}

// Lever arm d = x - x_p (minimum image, taken in FP64) and particle velocity
// at the cell centre (eq. 20) in FP64 (FP64 storage).
__device__ __forceinline__ void slot_geometry64(int c, double cxc, double cyc, double czc, double Lx, double hLx,
                                                double Ly, double hLy, double Lz, double hLz, const double* px,
                                                const double* py, const double* pz, const double* ux,
                                                const double* uy, const double* uz, const double* ox,
                                                const double* oy, const double* oz, double& dx, double& dy,
                                                double& dz, double& Vx, double& Vy, double& Vz) {
    dx = min_image(cxc - px[c], Lx, hLx);
    dy = min_image(cyc - py[c], Ly, hLy);
    dz = min_image(czc - pz[c], Lz, hLz);
    Vx = ux[c] + (oy[c] * dz - oz[c] * dy);
    Vy = uy[c] + (oz[c] * dx - ox[c] * dz);
    Vz = uz[c] + (ox[c] * dy - oy[c] * dx);
}

// Minimum image in FP32 of a displacement that is within a few box lengths.
__device__ __forceinline__ float wrap32(float t, float L, float invL) { return fmar(-L, __builtin_rintf(t * invL), t); }

// Waves per SIMD the register budget of the step kernel is cut for: 3 for
// FP64 storage (168 VGPRs), 4 for the deviation forms (128 VGPRs).
#ifndef PSM_WAVES_PER_EU
#define PSM_WAVES_PER_EU 3
#endif
#ifndef PSM_WAVES_PER_EU_DEV
#define PSM_WAVES_PER_EU_DEV 4
#endif
// Pull order of the step kernel (measured per storage form): the FP32 form
// pulls the next cell's values while it works on the current one; FP64 issues
// each cell's pulls before its mapping (not with the candidate filter, whose
// registers that would spill); FP16 pulls after the mapping (earlier or ahead
// was slower there).
#ifndef PSM_PREFETCH_F32
#define PSM_PREFETCH_F32 1
#endif
#ifndef PSM_PREFETCH_F16
#define PSM_PREFETCH_F16 0
#endif
#ifndef PSM_EARLY_PULLS_F64
#define PSM_EARLY_PULLS_F64 1
#endif
#ifndef PSM_EARLY_PULLS_F16
#define PSM_EARLY_PULLS_F16 0
#endif

// pull of the 19 values of one cell from the source planes z (rz), z-1 (rm)
// and z+1 (rp); direction q lies q * QB bytes into a block
#define PSM_LOAD19(F, rz, rm, rp)            \
    do {                                     \
        F[0] = S::ld(rz, o00, 0 * QB);       \
        F[1] = S::ld(rz, om0, 1 * QB);       \
        F[2] = S::ld(rz, op0, 2 * QB);       \
        F[3] = S::ld(rz, o0m, 3 * QB);       \
        F[4] = S::ld(rz, o0p, 4 * QB);       \
        F[5] = S::ld(rm, o00, 5 * QB);       \
        F[6] = S::ld(rp, o00, 6 * QB);       \
        F[7] = S::ld(rz, omm, 7 * QB);       \
        F[8] = S::ld(rz, opp, 8 * QB);       \
        F[9] = S::ld(rz, omp, 9 * QB);       \
        F[10] = S::ld(rz, opm, 10 * QB);     \
        F[11] = S::ld(rm, om0, 11 * QB);     \
        F[12] = S::ld(rp, op0, 12 * QB);     \
        F[13] = S::ld(rp, om0, 13 * QB);     \
        F[14] = S::ld(rm, op0, 14 * QB);     \
        F[15] = S::ld(rm, o0m, 15 * QB);     \
        F[16] = S::ld(rp, o0p, 16 * QB);     \
        F[17] = S::ld(rp, o0m, 17 * QB);     \
        F[18] = S::ld(rm, o0p, 18 * QB);     \
    } while (0)

template <class S, int MAP, bool FILT>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(S::DEV ? PSM_WAVES_PER_EU_DEV : PSM_WAVES_PER_EU, 8))) void k_psm_step(
    StepParams kp) {
    using R = typename S::R;
    using T = typename S::T;

    __shared__ double s_px[MAXC], s_py[MAXC], s_pz[MAXC], s_pr[MAXC], s_pfr[MAXC];
    __shared__ double s_ux[MAXC], s_uy[MAXC], s_uz[MAXC], s_ox[MAXC], s_oy[MAXC], s_oz[MAXC];
    // FP32 copies: centre relative to the tile centre (minimum image), the
    // squared reach of the overlap test with a rounding margin, and (for the
    // deviation forms) the velocities
    __shared__ float s_qx[MAXC], s_qy[MAXC], s_qz[MAXC], s_lim2[MAXC], s_rf[MAXC], s_frf[MAXC];
    __shared__ float s_uf[6][MAXC];
    __shared__ int s_pid[MAXC], s_slot[MAXC];
    __shared__ double s_acc[NWAVE][6][MAXC];
    __shared__ unsigned long long s_cmask[NWAVE][TZ_MAX];

    const int tid = threadIdx.x;
    const int TX = kp.tx, TY = kp.ty, TZ = kp.tz;
    const int lx = tid % TX, ly = tid / TX;
    const int wave = tid >> 6, lane = tid & 63;

    // XCD-aware persistent schedule: workgroup b runs on die b % 8; each die
    // walks one contiguous eighth of the tile list so that x-neighbouring
    // tiles (which share the cache lines of the shifted pulls) meet in the
    // same L2.
    const int G = gridDim.x;
    const int xcd = blockIdx.x % NXCD;
    const int gx8 = (G - xcd + NXCD - 1) / NXCD;
    const int m = blockIdx.x / NXCD;
    const int t_begin = (int)(((long long)kp.T_total * xcd) / NXCD);
    const int t_end = (int)(((long long)kp.T_total * (xcd + 1)) / NXCD);

    const PSM_CONST BoxDev* boxes = cptr(kp.boxes);
    const PSM_CONST int* tile_off = cptr(kp.tile_off);

    // Tile order: with a queue (persistent grid), the workgroups of a die take
    // the next tile of its eighth from that die's counter as they finish one;
    // otherwise workgroup m of a die takes tiles m, m + gx8, ...
    __shared__ int s_next;
    int* const queue = kp.queue;
    int t = t_begin + m;
    if (queue) {
        if (tid == 0) s_next = t_begin + atomicAdd(queue + xcd, 1);
        __syncthreads();
        t = s_next;
    }
    while (t < t_end) {
        int b = 0;
        if (kp.nbox > 1) {
            const PSM_CONST int* tb = cptr(kp.box_tile_base);
            int lo = 0, hi = kp.nbox - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (tb[mid] <= t) lo = mid; else hi = mid - 1;
            }
            b = lo;
        }
        const PSM_CONST BoxDev& bx = boxes[b];
        const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
        // MAP = 1 instantiates the sampling path for contexts in which any box
        // samples; each box still uses its own mapping
        const bool lin_map = MAP == 0 || bx.mapping == 0;
        const int ntx = bx.ntx, nty = bx.nty;
        const int lt = t - bx.tile_base;
        const int tcx = lt % ntx;
        const int tcy = (lt / ntx) % nty;
        const int tcz = lt / (ntx * nty);
        const int e0 = tile_off[t];
        const int nc = tile_off[t + 1] - e0;   // at most MAXC: the scan caps every list
        const double Lx = bx.L[0], Ly = bx.L[1], Lz = bx.L[2];
        const double hLx = bx.halfL[0], hLy = bx.halfL[1], hLz = bx.halfL[2];
        // tile centre in cell coordinates
        const double tmx = tcx * TX + 0.5 * TX, tmy = tcy * TY + 0.5 * TY, tmz = tcz * TZ + 0.5 * TZ;

        if (nc > 0) {
            for (int c = tid; c < nc; c += WG) {
                int p = kp.tile_pid[e0 + c];
                s_pid[c] = p;
                s_slot[c] = kp.tile_slot[e0 + c];
                const double px = kp.P.x[p], py = kp.P.y[p], pz = kp.P.z[p], pr = kp.P.r[p], pfr = kp.P.fr[p];
                s_px[c] = px; s_py[c] = py; s_pz[c] = pz;
                s_pr[c] = pr; s_pfr[c] = pfr;
                s_qx[c] = (float)min_image(px - tmx, Lx, hLx);
                s_qy[c] = (float)min_image(py - tmy, Ly, hLy);
                s_qz[c] = (float)min_image(pz - tmz, Lz, hLz);
                const double lim = pr + (lin_map ? pfr : bx.reach) + bx.margin32;
                s_lim2[c] = (float)(lim * lim);
                s_rf[c] = (float)pr;
                s_frf[c] = (float)pfr;
                const double u[6] = {kp.P.ux[p], kp.P.uy[p], kp.P.uz[p], kp.P.ox[p], kp.P.oy[p], kp.P.oz[p]};
                s_ux[c] = u[0]; s_uy[c] = u[1]; s_uz[c] = u[2];
                s_ox[c] = u[3]; s_oy[c] = u[4]; s_oz[c] = u[5];
#pragma unroll
                for (int k = 0; k < 6; ++k) s_uf[k][c] = (float)u[k];
            }
            for (int i = tid; i < NWAVE * 6 * MAXC; i += WG) (&s_acc[0][0][0])[i] = 0.0;
        }
        __syncthreads();

        const int x = tcx * TX + lx;
        const int y = tcy * TY + ly;
        const bool lane_ok = (x < nx) && (y < ny);
        const int xs = lane_ok ? x : 0, ys = lane_ok ? y : 0;
        const int xm = xs == 0 ? nx - 1 : xs - 1, xp = xs == nx - 1 ? 0 : xs + 1;
        const int ym = ys == 0 ? ny - 1 : ys - 1, yp = ys == ny - 1 ? 0 : ys + 1;
        // byte offsets inside a z-plane of the nine (x, y) source columns;
        // they do not depend on z (a plane holds fewer than 2^31 bytes)
        const int pitch = bx.pitch;
        auto inplane = [pitch](int xx, int yy) -> unsigned {
            int c = xx + pitch * yy;
            return (unsigned)(((c / BLK) * (NQ * BLK) + (c % BLK)) * (int)sizeof(T));
        };
        // lanes next to a resting side wall (x = 0, nx - 1; y = 0, ny - 1): bits 0-3
        const int edge = !lane_ok || !bx.walls_xy ? 0
                         : (((bx.walls_xy & 1) && xs == 0) ? 1 : 0) | (((bx.walls_xy & 1) && xs == nx - 1) ? 2 : 0) |
                               (((bx.walls_xy & 2) && ys == 0) ? 4 : 0) | (((bx.walls_xy & 2) && ys == ny - 1) ? 8 : 0);
        const bool edge_wave = __ballot(edge != 0) != 0ull;
        const unsigned o00 = inplane(xs, ys), om0 = inplane(xm, ys), op0 = inplane(xp, ys);
        const unsigned o0m = inplane(xs, ym), o0p = inplane(xs, yp);
        const unsigned omm = inplane(xm, ym), opp = inplane(xp, yp), omp = inplane(xm, yp), opm = inplane(xp, ym);
        const long long pbytes = bx.plane_elems * (long long)sizeof(T);
        const unsigned pb32 = (unsigned)pbytes;
        const char* src = (const char*)bx.grid[kp.parity];
        const char* dst = (const char*)bx.grid[kp.parity ^ 1];
        const R omega = pick<R>(bx.omega, bx.omega_f);
        const R om1 = pick<R>(bx.om1, bx.om1_f);
        const R gx = pick<R>(bx.g[0], bx.g_f[0]), gy = pick<R>(bx.g[1], bx.g_f[1]), gz = pick<R>(bx.g[2], bx.g_f[2]);
        // scaled storage (FP16): the kernel works on s d; the quadratic terms
        // carry 1/s and every particle velocity is multiplied by s
        const R sc = S::SCALED ? (R)kp.h_scale : (R)1;
        const R k15 = pick<R>(bx.k15, bx.k15_f);
        const R k45 = pick<R>(bx.k45, bx.k45_f);
        const double cxc = xs + 0.5, cyc = ys + 0.5;
        // this cell's centre relative to the tile centre (FP32, exact)
        const float rx = (float)(lx + 0.5 - 0.5 * TX), ry = (float)(ly + 0.5 - 0.5 * TY);
        const float Lxf = (float)Lx, Lyf = (float)Ly, Lzf = (float)Lz;
        const float iLx = 1.0f / Lxf, iLy = 1.0f / Lyf, iLz = 1.0f / Lzf;
        // Candidate filter: bit c of s_cmask[wave][k] is set if candidate c
        // can reach a cell of this wave at the tile's k-th z: the distance from
        // the sphere centre to the rectangle of the wave's cell centres (lanes
        // past the box edge only enlarge it) is below r + f(r), or r + the
        // sampling reach, plus a margin that covers the FP32 rounding of the
        // test. Other candidates give zero fraction to all of those cells.
        if (FILT && nc > 0) {
            float xy2 = 0.0f, pz = 0.0f, lim2 = -1.0f;
            if (lane < nc) {
                const int wwx = TX < 64 ? TX : 64, wwy = TX < 64 ? 64 / TX : 1;
                const int wx0 = tcx * TX + (64 * wave) % TX, wy0 = tcy * TY + (64 * wave) / TX;
                double ex = fabs(min_image(wx0 + 0.5 * wwx - s_px[lane], bx.L[0], bx.halfL[0])) - 0.5 * (wwx - 1);
                double ey = fabs(min_image(wy0 + 0.5 * wwy - s_py[lane], bx.L[1], bx.halfL[1])) - 0.5 * (wwy - 1);
                ex = ex > 0.0 ? ex : 0.0;
                ey = ey > 0.0 ? ey : 0.0;
                xy2 = (float)(ex * ex + ey * ey);
                pz = (float)s_pz[lane];
                const double lim = s_pr[lane] + (lin_map ? s_pfr[lane] : bx.reach) + 0.05;
                lim2 = (float)(lim * lim);
            }
            const float fnz = (float)nz;
            for (int k = 0; k < TZ; ++k) {
                float ez = (float)(tcz * TZ + k) + 0.5f - pz;
                ez = ez >= 0.5f * fnz ? ez - fnz : (ez < -0.5f * fnz ? ez + fnz : ez);
                const unsigned long long m = __ballot(xy2 + ez * ez < lim2);
                if (lane == 0) s_cmask[wave][k] = m;
            }
        }

        constexpr int QB = BLK * (int)sizeof(T);

        // Latency hiding: PREF pulls the next cell's 19 values (one cell up in
        // z) while the current one is mapped and collided; EARLY issues the
        // current cell's pulls before its mapping.
        constexpr bool PREF = S::DEV && !FILT && (S::SCALED ? PSM_PREFETCH_F16 : PSM_PREFETCH_F32);
        constexpr bool EARLY = !PREF && !FILT && (S::DEV ? (S::SCALED && PSM_EARLY_PULLS_F16) : PSM_EARLY_PULLS_F64);
        R fn[NQ];
        if constexpr (PREF) {
            const int z0 = tcz * TZ;
            if (lane_ok && z0 < nz) {
                const int zm0 = z0 == 0 ? nz - 1 : z0 - 1, zp0 = z0 == nz - 1 ? 0 : z0 + 1;
                const Rsrc a = plane_rsrc(src + z0 * pbytes, pb32), am = plane_rsrc(src + zm0 * pbytes, pb32),
                           ap = plane_rsrc(src + zp0 * pbytes, pb32);
                PSM_LOAD19(fn, a, am, ap);
            }
        }

        for (int k = 0; k < TZ; ++k) {
            const int z = tcz * TZ + k;
            if (z >= nz) break;
            const double czc = z + 0.5;
            const float rz = (float)(k + 0.5 - 0.5 * TZ);
            const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
            // buffer resources of the source planes z, z-1, z+1 and the
            // destination plane z
            const Rsrc sz = plane_rsrc(src + z * pbytes, pb32);
            const Rsrc sm = plane_rsrc(src + zm * pbytes, pb32);
            const Rsrc sp = plane_rsrc(src + zp * pbytes, pb32);
            const Rsrc dz_ = plane_rsrc(dst + z * pbytes, pb32);

            // 2a. pull: f_q(x) = grid[q][x - c_q] (eq. 2 read backwards)
            R f[NQ];
            if constexpr (PREF) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) f[q] = fn[q];
                const int z1 = z + 1;
                if (lane_ok && k + 1 < TZ && z1 < nz) {
                    // planes z + 1 (own), z (below) and z + 2 (above, periodic)
                    const Rsrc a2 = plane_rsrc(src + (z1 == nz - 1 ? 0 : z1 + 1) * pbytes, pb32);
                    PSM_LOAD19(fn, sp, sz, a2);
                }
            } else if constexpr (EARLY) {
                if (lane_ok) PSM_LOAD19(f, sz, sm, sp);
            }

            // 1. solid fractions of this cell from the staged candidates (Sec. 2.3.2);
            // with the filter, only the candidates that can reach this wave at this z.
            // The fraction is FP64, bit for bit that of the read-out path, except
            // that the FP16 form takes the linear approximation in FP32.
            int c0 = -1, c1 = -1;
            double B0 = 0.0, B1 = 0.0;
            int dropped = 0;   // overlaps beyond the two slots at this cell
#define PSM_MAP_ONE(c)                                                                                       \
    do {                                                                                                    \
        bool near_ = true;                                                                                  \
        if constexpr (S::DEV) {                                                                             \
            const float tx_ = wrap32(rx - s_qx[c], Lxf, iLx);                                               \
            const float ty_ = wrap32(ry - s_qy[c], Lyf, iLy);                                               \
            const float tz_ = wrap32(rz - s_qz[c], Lzf, iLz);                                               \
            const float d2_ = fmar(tz_, tz_, fmar(ty_, ty_, tx_ * tx_));                                    \
            near_ = d2_ <= s_lim2[c];                                                                       \
            if (S::SCALED && near_ && lin_map) {                                                            \
                /* FP16 storage: linear approximation of eq. (26) in FP32 (its error, about */              \
                /* 1e-6 of a cell, is far below the FP16 rounding of the stored values) */                  \
                const float eps_ = s_frf[c] - (__builtin_amdgcn_sqrtf(d2_) - s_rf[c]);                       \
                if (eps_ > 0.0f) slots_insert(sl, c, s_pid[c], (double)(eps_ < 1.0f ? eps_ : 1.0f));         \
                near_ = false;                                                                              \
            }                                                                                               \
        }                                                                                                   \
        if (near_) {                                                                                        \
            double dx = min_image(cxc - s_px[c], Lx, hLx);                                                  \
            double dy = min_image(cyc - s_py[c], Ly, hLy);                                                  \
            double dz = min_image(czc - s_pz[c], Lz, hLz);                                                  \
            double B = lin_map ? overlap_linear(dx, dy, dz, s_pr[c], s_pfr[c])                              \
                               : overlap_subsample(dx, dy, dz, s_pr[c], bx.nsub, bx.sub_off, bx.reach);     \
            if (B > 0.0) slots_insert(sl, c, s_pid[c], B);                                                  \
        }                                                                                                   \
    } while (0)
            if constexpr (FILT) {
                unsigned long long cm = nc > 0 ? s_cmask[wave][k] : 0ull;
                // wave-uniform: keep the mask and its loop in scalar registers
                cm = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(cm >> 32)) << 32) |
                     (unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)cm);
                if (cm != 0ull) {
                    Slots sl;
                    slots_init(sl);
                    if (lane_ok) {
                        while (cm != 0ull) {
                            const int c = __ffsll((long long)cm) - 1;
                            cm &= cm - 1ull;
                            PSM_MAP_ONE(c);
                        }
                        slots_finish(sl);
                    }
                    c0 = sl.c0; c1 = sl.c1; B0 = sl.B0; B1 = sl.B1; dropped = sl.dropped;
                }
            } else if (nc > 0) {
                Slots sl;
                slots_init(sl);
                if (lane_ok) {
                    for (int c = 0; c < nc; ++c) PSM_MAP_ONE(c);
                    slots_finish(sl);
                }
                c0 = sl.c0; c1 = sl.c1; B0 = sl.B0; B1 = sl.B1; dropped = sl.dropped;
            }
#undef PSM_MAP_ONE
            const bool psm_wave = __ballot(c0 >= 0) != 0ull;
            // a third overlap is dropped (the two strongest slots stay) and flagged
            // once per wave; the host reports it in strict-slot mode
            if (psm_wave && __ballot(dropped != 0) != 0ull && lane == 0) atomicOr(kp.flags, FLAG_SLOT_OVERFLOW);

            // 2b. boundaries of the pulled values
            R hx = 0, hy = 0, hz = 0;   // 2 j - U, for the force of eq. (21)
            if (lane_ok) {
                // through a face (first and last z plane of a box with walls):
                // the population this cell sent against it last step, by the
                // face rule; computed before the pulls so that its
                // temporaries are not live beside them (uniform branches)
                const bool face_plane = bx.walls && (z == 0 || z == nz - 1);
                R fb[5] = {0, 0, 0, 0, 0};
                if (face_plane) {
                    const int w = z == 0 ? 0 : 1;
                    // entering directions through this face and their opposites
                    constexpr int in0[5] = {5, 11, 14, 15, 18}, in1[5] = {6, 12, 13, 16, 17};
                    if (bx.face_type[w] == FACE_VELOCITY) {
                        const R ws = S::SCALED ? sc : (R)1;
#pragma unroll
                        for (int i = 0; i < 5; ++i) {
                            const int q = w == 0 ? in0[i] : in1[i];
                            fb[i] = S::ld(sz, o00, inv_dir(q) * QB) + ws * (R)bx.bw[w][q];
                        }
                    } else {
                        // anti-bounce-back with the cell's post-collision velocity
                        // (its own 19 slots); deviation units carry rho_w - 1
                        R ux = 0, uy = 0, uz = 0;
#pragma unroll
                        for (int q = 1; q < NQ; ++q) {
                            const R v = S::ld(sz, o00, q * QB);
                            ux += (R)CX[q] * v; uy += (R)CY[q] * v; uz += (R)CZ[q] * v;
                        }
                        const R rw = S::DEV ? (R)(bx.face_rho[w] - 1.0) * sc : (R)bx.face_rho[w];
                        const R uu = k15 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
                        for (int i = 0; i < 5; ++i) {
                            const int q = w == 0 ? in0[i] : in1[i];
                            const R cu = (R)CX[q] * ux + (R)CY[q] * uy + (R)CZ[q] * uz;
                            fb[i] = (R)(2.0 * wq(q)) * (rw + k45 * (cu * cu) - uu) - S::ld(sz, o00, inv_dir(q) * QB);
                        }
                    }
                }
                if constexpr (!PREF && !EARLY) PSM_LOAD19(f, sz, sm, sp);
                if (face_plane) {
                    if (z == 0) {
                        f[5] = fb[0]; f[11] = fb[1]; f[14] = fb[2]; f[15] = fb[3]; f[18] = fb[4];
                    } else {
                        f[6] = fb[0]; f[12] = fb[1]; f[13] = fb[2]; f[16] = fb[3]; f[17] = fb[4];
                    }
                }
                if (edge_wave && edge) {
                    // resting side walls (they win over a z face): a population
                    // pulled from behind a wall is the one this cell sent
                    // against it last step
#pragma unroll
                    for (int q = 1; q < NQ; ++q) {
                        const bool hit = (CX[q] == 1 && (edge & 1)) || (CX[q] == -1 && (edge & 2)) ||
                                         (CY[q] == 1 && (edge & 4)) || (CY[q] == -1 && (edge & 8));
                        if (hit) f[q] = S::ld(sz, o00, inv_dir(q) * QB);
                    }
                }

                // 3. moments, eqs. (6)-(7), accumulated from the sum and the
                // difference of each inverse pair (q, q+1), q = 2k-1 with c_q =
                // +x, +y, +z, (1,1,0), (1,-1,0), (1,0,1), (1,0,-1), (0,1,1),
                // (0,1,-1) for k = 1..9; U carries the f/2 shift
                R rho = f[0], jx, jy, jz;
                {
                    R d;
                    rho += f[1] + f[2]; jx = f[1] - f[2];
                    rho += f[3] + f[4]; jy = f[3] - f[4];
                    rho += f[5] + f[6]; jz = f[5] - f[6];
                    rho += f[7] + f[8]; d = f[7] - f[8]; jx += d; jy += d;
                    rho += f[9] + f[10]; d = f[9] - f[10]; jx += d; jy -= d;
                    rho += f[11] + f[12]; d = f[11] - f[12]; jx += d; jz += d;
                    rho += f[13] + f[14]; d = f[13] - f[14]; jx += d; jz -= d;
                    rho += f[15] + f[16]; d = f[15] - f[16]; jy += d; jz += d;
                    rho += f[17] + f[18]; d = f[17] - f[18]; jy += d; jz -= d;
                }
                const R half = (R)0.5;
                const R Ux = fmar(half, sc * gx, jx), Uy = fmar(half, sc * gy, jy), Uz = fmar(half, sc * gz, jz);
                const R uu = fmar(Uz, Uz, fmar(Uy, Uy, Ux * Ux));
                const R base = fmar(-k15, uu, rho);
                const R Ug3 = (R)3.0 * fmar(Uz, gz, fmar(Uy, gy, Ux * gx));
                const R pu0 = pick<R>(bx.pw[0], bx.pw_f[0]) * Ug3;
                WClass<R> w1, w2;
                {
                    constexpr R W1r = (R)W1, W2r = (R)W2;
                    w1.Wb = W1r * base; w2.Wb = W2r * base;
                    w1.W3 = (R)3 * W1r; w2.W3 = (R)3 * W2r;
                    w1.Wk = pick<R>(bx.wk[1], bx.wk_f[1]); w2.Wk = pick<R>(bx.wk[2], bx.wk_f[2]);
                    w1.owk = pick<R>(bx.owk[1], bx.owk_f[1]); w2.owk = pick<R>(bx.owk[2], bx.owk_f[2]);
                    w1.ow3 = pick<R>(bx.ow3[1], bx.ow3_f[1]); w2.ow3 = pick<R>(bx.ow3[2], bx.ow3_f[2]);
                    w1.owb_pu = fmar(omega, w1.Wb, -pick<R>(bx.pw[1], bx.pw_f[1]) * Ug3);
                    w2.owb_pu = fmar(omega, w2.Wb, -pick<R>(bx.pw[2], bx.pw_f[2]) * Ug3);
                }
#define PSM_FA(Q) pick<R>(S::SCALED ? bx.fa_scaled[Q / 2] : bx.fa[Q / 2], S::SCALED ? bx.fa_scaled_f[Q / 2] : bx.fa_f[Q / 2])
#define PSM_FS(Q) pick<R>(bx.fs[Q / 2], bx.fs_f[Q / 2])
#define PSM_STORE(Q) S::st(dz_, o00, (Q) * QB, f[Q])

                // 4. collision; each pair is stored as soon as it is final
                if (!psm_wave) {
                    f[0] = fmar(om1, f[0], fmar(omega * (R)W0, base, -pu0));
                    PSM_STORE(0);
#define PSM_PAIR(Q)                                                                                 \
    pair_fluid<R, Q>(f[Q], f[Q + 1], cdot<R, Q>(Ux, Uy, Uz), Q < 7 ? w1 : w2, PSM_FA(Q), PSM_FS(Q), om1); \
    PSM_STORE(Q);                                                                                   \
    PSM_STORE(Q + 1)
                    PSM_PAIR(1); PSM_PAIR(3); PSM_PAIR(5); PSM_PAIR(7); PSM_PAIR(9);
                    PSM_PAIR(11); PSM_PAIR(13); PSM_PAIR(15); PSM_PAIR(17);
#undef PSM_PAIR
                } else {
                    hx = (R)2 * jx - Ux; hy = (R)2 * jy - Uy; hz = (R)2 * jz - Uz;
                    // slot terms with U_p(x) of eq. (20) (times the storage scale)
                    // (a wave with a slot somewhere: lanes without one add nothing)
                    R Bt = 0, A0 = 0, Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0, Px = 0, Py = 0, Pz = 0;
#pragma unroll
                    for (int sl = 0; sl < 2; ++sl) {
                        const int c = sl == 0 ? c0 : c1;
                        if (c < 0) continue;   // slot 1 is only filled after slot 0
                        R Vx, Vy, Vz;
                        if constexpr (S::DEV) {
                            // lever arm from the FP32 tile-relative centre
                            const float dx = wrap32(rx - s_qx[c], Lxf, iLx);
                            const float dy = wrap32(ry - s_qy[c], Lyf, iLy);
                            const float dz = wrap32(rz - s_qz[c], Lzf, iLz);
                            Vx = sc * (s_uf[0][c] + (s_uf[4][c] * dz - s_uf[5][c] * dy));
                            Vy = sc * (s_uf[1][c] + (s_uf[5][c] * dx - s_uf[3][c] * dz));
                            Vz = sc * (s_uf[2][c] + (s_uf[3][c] * dy - s_uf[4][c] * dx));
                        } else {
                            double dx, dy, dz;
                            slot_geometry64(c, cxc, cyc, czc, Lx, hLx, Ly, hLy, Lz, hLz, s_px, s_py, s_pz, s_ux,
                                            s_uy, s_uz, s_ox, s_oy, s_oz, dx, dy, dz, Vx, Vy, Vz);
                        }
                        const R Bs = (R)(sl == 0 ? B0 : B1);
                        const R qx = Bs * Vx, qy = Bs * Vy, qz = Bs * Vz;
                        const R a0 = Bs * fmar(-k15, fmar(Vz, Vz, fmar(Vy, Vy, Vx * Vx)), rho);
                        if (sl == 0) {
                            Bt = Bs; A0 = a0; Px = qx; Py = qy; Pz = qz;
                            Mxx = qx * Vx; Myy = qy * Vy; Mzz = qz * Vz;
                            Mxy = qx * Vy; Mxz = qx * Vz; Myz = qy * Vz;
                        } else {
                            Bt = Bt + Bs; A0 = A0 + a0;
                            Px = Px + qx; Py = Py + qy; Pz = Pz + qz;
                            Mxx = fmar(qx, Vx, Mxx); Myy = fmar(qy, Vy, Myy); Mzz = fmar(qz, Vz, Mzz);
                            Mxy = fmar(qx, Vy, Mxy); Mxz = fmar(qx, Vz, Mxz); Myz = fmar(qy, Vz, Myz);
                        }
                    }
                    const R omB = (R)1 - Bt;
                    const R Mxy2 = Mxy + Mxy, Mxz2 = Mxz + Mxz, Myz2 = Myz + Myz;
                    const R omw = omB * omega;
                    const R alpha = ((R)1 - Bt) - omw, beta = omw - Bt, gamma = omw + Bt;
                    const R pu1 = pick<R>(bx.pw[1], bx.pw_f[1]) * Ug3, pu2 = pick<R>(bx.pw[2], bx.pw_f[2]) * Ug3;
                    const R C11 = fmar(beta, w1.Wb, fmar(-omB, pu1, (R)W1 * A0));
                    const R C12 = fmar(beta, w2.Wb, fmar(-omB, pu2, (R)W2 * A0));
                    const R C21 = beta * w1.Wk, C22 = beta * w2.Wk;
                    const R C31 = gamma * w1.W3, C32 = gamma * w2.W3;
                    // rest population: c = 0, qbar = q
                    f[0] = fmar(alpha + Bt, f[0], fmar(beta * (R)W0, base, fmar(-omB, pu0, (R)W0 * A0)));
                    PSM_STORE(0);
#define PSM_PAIR(Q)                                                                                              \
    pair_psm<R, Q>(f[Q], f[Q + 1], cdot<R, Q>(Ux, Uy, Uz), Q < 7 ? C11 : C12, Q < 7 ? C21 : C22, Q < 7 ? C31 : C32, \
                   Q < 7 ? w1.Wk : w2.Wk, Q < 7 ? w1.W3 : w2.W3, omB * PSM_FS(Q), omB * PSM_FA(Q), alpha, Bt,        \
                   cmc<R, Q>(Mxx, Myy, Mzz, Mxy2, Mxz2, Myz2), cdot<R, Q>(Px, Py, Pz));                             \
    PSM_STORE(Q);                                                                                                \
    PSM_STORE(Q + 1)
                    PSM_PAIR(1); PSM_PAIR(3); PSM_PAIR(5); PSM_PAIR(7); PSM_PAIR(9);
                    PSM_PAIR(11); PSM_PAIR(13); PSM_PAIR(15); PSM_PAIR(17);
#undef PSM_PAIR
                }
#undef PSM_STORE
#undef PSM_FA
#undef PSM_FS
            }

            // 5. force and torque of eqs. (21)-(22): sum_q C^solid_{q,s} c_qbar
            // = 2 j - U - U_p(x) per slot (first moment of eq. 19); per-sphere
            // wave sums accumulated per wave in LDS in FP64 in a fixed order.
            // The deviation forms compute each cell's share and the wave sum in
            // FP32 (the collision's precision); FP64 storage does both in FP64.
            if (psm_wave) {
                int pend0 = lane_ok ? c0 : -1, pend1 = lane_ok ? c1 : -1;
                while (true) {
                    unsigned long long live = __ballot(pend0 >= 0 || pend1 >= 0);
                    if (live == 0ull) break;
                    int leader = __ffsll((long long)live) - 1;
                    int mine = pend0 >= 0 ? pend0 : pend1;
                    // the leader's candidate, read into a scalar register
                    const int c = __builtin_amdgcn_readlane(mine, leader);
                    double Bs = 0.0;
                    if (pend0 == c) { Bs = B0; pend0 = -1; }
                    else if (pend1 == c) { Bs = B1; pend1 = -1; }
                    R v[6] = {0, 0, 0, 0, 0, 0};
                    if (Bs != 0.0) {
                        R dx, dy, dz, Vx, Vy, Vz;
                        if constexpr (S::DEV) {
                            dx = wrap32(rx - s_qx[c], Lxf, iLx);
                            dy = wrap32(ry - s_qy[c], Lyf, iLy);
                            dz = wrap32(rz - s_qz[c], Lzf, iLz);
                            Vx = sc * (s_uf[0][c] + (s_uf[4][c] * dz - s_uf[5][c] * dy));
                            Vy = sc * (s_uf[1][c] + (s_uf[5][c] * dx - s_uf[3][c] * dz));
                            Vz = sc * (s_uf[2][c] + (s_uf[3][c] * dy - s_uf[4][c] * dx));
                        } else {
                            slot_geometry64(c, cxc, cyc, czc, Lx, hLx, Ly, hLy, Lz, hLz, s_px, s_py, s_pz, s_ux,
                                            s_uy, s_uz, s_ox, s_oy, s_oz, dx, dy, dz, Vx, Vy, Vz);
                        }
                        const R Bh = (R)(S::SCALED ? Bs * (double)kp.h_inv : Bs);
                        const R fx = Bh * (hx - Vx), fy = Bh * (hy - Vy), fz = Bh * (hz - Vz);
                        v[0] = fx;
                        v[1] = fy;
                        v[2] = fz;
                        v[3] = dy * fz - dz * fy;
                        v[4] = dz * fx - dx * fz;
                        v[5] = dx * fy - dy * fx;
                    }
                    const R sum = wave_sum6<R>(v, lane);
                    if (lane < 6) s_acc[wave][lane][c] += (double)sum;
                }
            }
        }

        __syncthreads();
        if (nc > 0) {
            for (int i = tid; i < nc * 6; i += WG) {
                int c = i / 6, k6 = i - 6 * c;
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < NWAVE; ++w) s += s_acc[w][k6][c];
                kp.partial[(long long)s_slot[c] * 6 + k6] = s;
            }
        }
        __syncthreads();
        // every thread has read s_next before the barriers of this tile
        if (queue) {
            if (tid == 0) s_next = t_begin + atomicAdd(queue + xcd, 1);
            __syncthreads();
            t = s_next;
        } else {
            t += gx8;
        }
    }
}

// ---------------------------------------------------------------------------
// Per-sphere force/torque: sum the tile partials of every tile of the
// sphere's bounding box, in a fixed tile order (deterministic).
// One 64-wide wave per sphere: lane l takes the sphere's tiles l, l+64, ...
// (in the fixed bounding-box order), then a fixed butterfly adds the lanes.
__global__ __launch_bounds__(256) void k_reduce_forces(ReduceParams rp) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= rp.P_total) return;   // whole wave leaves together
    const int b = rp.part_box[p];
    const BoxDev& bx = rp.boxes[b];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (p - bx.part_base < bx.np) {
        int lo, hi;
        aabb_cells(rp.P.x[p], rp.P.r[p], lo, hi);
        AxisTiles ax = axis_tiles(lo, hi, bx.nx, rp.ts.tx, bx.ntx);
        aabb_cells(rp.P.y[p], rp.P.r[p], lo, hi);
        AxisTiles ay = axis_tiles(lo, hi, bx.ny, rp.ts.ty, bx.nty);
        aabb_cells(rp.P.z[p], rp.P.r[p], lo, hi);
        AxisTiles az = axis_tiles(lo, hi, bx.nz, rp.ts.tz, bx.ntz);
        const int ntot = ax.count() * ay.count() * az.count();
        // the sphere's slots: one per tile of its bounding box, in that order
        const double* pp = rp.partial + ((long long)bx.pbase + (long long)(p - bx.part_base) * bx.pstride) * 6;
        for (int k = lane; k < ntot; k += 64) {
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] += pp[(long long)k * 6 + c];
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double v = wave_sum(acc[c]);
        if (lane == 0) rp.P.acc[(long long)p * 6 + c] = v;
    }
}

// ---------------------------------------------------------------------------
// Tile binning (the paper's sub-block particle lists, built on the device):
// count -> exclusive scan -> fill.
// One 64-wide wave per sphere; its lanes walk the bounding box's tiles.
template <bool FILL>
__global__ __launch_bounds__(256) void k_bin(BinParams bp) {
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= bp.P_total) return;
    const int b = bp.part_box[p];
    const BoxDev& bx = bp.boxes[b];
    if (p - bx.part_base >= bx.np) return;
    int lo, hi;
    aabb_cells(bp.P.x[p], bp.P.r[p], lo, hi);
    AxisTiles ax = axis_tiles(lo, hi, bx.nx, bp.ts.tx, bx.ntx);
    aabb_cells(bp.P.y[p], bp.P.r[p], lo, hi);
    AxisTiles ay = axis_tiles(lo, hi, bx.ny, bp.ts.ty, bx.nty);
    aabb_cells(bp.P.z[p], bp.P.r[p], lo, hi);
    AxisTiles az = axis_tiles(lo, hi, bx.nz, bp.ts.tz, bx.ntz);
    const int nxt = ax.count(), nyt = ay.count(), nzt = az.count();
    const int ntot = nxt * nyt * nzt;
    for (int k = lane; k < ntot; k += 64) {
        int kx = k % nxt, ky = (k / nxt) % nyt, kz = k / (nxt * nyt);
        int t = bx.tile_base + ax.at(kx) + bx.ntx * (ay.at(ky) + bx.nty * az.at(kz));
        if (!FILL) {
            atomicAdd(&bp.tile_cnt[t], 1);
        } else {
            // a list holds at most MAXC spheres (the scan caps it; the excess
            // is flagged from the uncapped maximum)
            int pos = atomicSub(&bp.tile_cnt[t], 1) - 1;
            long long e = (long long)bp.tile_off[t] + pos;
            const long long slot = (long long)bx.pbase + (long long)(p - bx.part_base) * bx.pstride + k;
            if (pos < MAXC && e < bp.cap) {
                bp.tile_pid[e] = p;
                bp.tile_slot[e] = (int)slot;
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) bp.partial[slot * 6 + c] = 0.0;
            }
        }
    }
}

__global__ void k_fill_int(int* a, long long n, int v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

// Exclusive scan of cnt[0..n) into off[0..n] in three passes over chunks of
// SCAN_CHUNK counts: chunk sums and maxima, a one-workgroup scan of the chunk
// sums, then each chunk scanned with its offset. Every list length is capped
// at MAXC; stats[0] = largest uncapped count, stats[1] = total of the lists.
constexpr int SCAN_CHUNK = 1024;

__device__ inline int block_incl_scan_256(int v, int* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        int add = tid >= d ? sh[tid - d] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    int r = sh[tid];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_scan_chunks(const int* cnt, int n, int* csum, int* cmax) {
    __shared__ int s_sum[256], s_max[256];
    const int tid = threadIdx.x;
    const int base = blockIdx.x * SCAN_CHUNK;
    int sum = 0, mx = 0;
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
        int i = base + k * 256 + tid;
        int v = i < n ? cnt[i] : 0;
        sum += v < MAXC ? v : MAXC;   // list lengths are capped at MAXC
        mx = v > mx ? v : mx;         // the uncapped maximum reports an excess
    }
    s_sum[tid] = sum;
    s_max[tid] = mx;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if (tid < d) {
            s_sum[tid] += s_sum[tid + d];
            s_max[tid] = s_max[tid] > s_max[tid + d] ? s_max[tid] : s_max[tid + d];
        }
        __syncthreads();
    }
    if (tid == 0) {
        csum[blockIdx.x] = s_sum[0];
        cmax[blockIdx.x] = s_max[0];
    }
}

__global__ __launch_bounds__(256) void k_scan_sums(int* csum, const int* cmax, int nchunk, int* stats) {
    __shared__ int sh[256];
    __shared__ int s_carry, s_max;
    const int tid = threadIdx.x;
    if (tid == 0) { s_carry = 0; s_max = 0; }
    __syncthreads();
    int mymax = 0;
    for (int base = 0; base < nchunk; base += 256) {
        int i = base + tid;
        int v = i < nchunk ? csum[i] : 0;
        mymax = (i < nchunk && cmax[i] > mymax) ? cmax[i] : mymax;
        int inc = block_incl_scan_256(v, sh);
        if (i < nchunk) csum[i] = s_carry + inc - v;   // exclusive offset of chunk i
        __syncthreads();
        if (tid == 255) s_carry += inc;
        __syncthreads();
    }
    atomicMax(&s_max, mymax);
    __syncthreads();
    if (tid == 0) {
        stats[0] = s_max;
        stats[1] = s_carry;
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(const int* cnt, int n, const int* coff, int* off,
                                                    const int* stats) {
    __shared__ int sh[256];
    const int tid = threadIdx.x;
    const int base = blockIdx.x * SCAN_CHUNK;
    // each thread owns 4 consecutive counts
    int v[4], loc = 0;
    for (int k = 0; k < 4; ++k) {
        int i = base + tid * 4 + k;
        v[k] = i < n ? (cnt[i] < MAXC ? cnt[i] : MAXC) : 0;
        loc += v[k];
    }
    int inc = block_incl_scan_256(loc, sh);
    int run = coff[blockIdx.x] + inc - loc;
    for (int k = 0; k < 4; ++k) {
        int i = base + tid * 4 + k;
        if (i < n) off[i] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) off[n] = stats[1];
}

// ---------------------------------------------------------------------------
// State I/O. Canonical f(x,t) = grid[q][x - c_q] (pull storage).

// Face crossed by a neighbour at z-index zz: -1 none (inside or periodic), 0 bottom, 1 top.
__device__ inline int face_of(const BoxDev& bx, int zz) {
    return !bx.walls ? -1 : (zz < 0 ? 0 : (zz >= bx.nz ? 1 : -1));
}

// True if the neighbour at (xx, yy) lies behind a resting side wall.
__device__ inline bool behind_side_wall(const BoxDev& bx, int xx, int yy) {
    return ((bx.walls_xy & 1) && (xx < 0 || xx >= bx.nx)) || ((bx.walls_xy & 2) && (yy < 0 || yy >= bx.ny));
}

// Post-collision velocity of a cell from its own 19 stored slots (slot q of
// cell x holds the value it sent in direction q), in S::to_f64 units.
template <class S>
__device__ inline void slot_velocity(const BoxDev& bx, const typename S::T* g, int x, int y, int z, float inv,
                                     double u[3]) {
    u[0] = u[1] = u[2] = 0.0;
    for (int q = 1; q < NQ; ++q) {
        double v = S::to_f64(g[pdf_index(bx, q, x, y, z)], inv);
        u[0] += v * CX[q]; u[1] += v * CY[q]; u[2] += v * CZ[q];
    }
}

// Anti-bounce-back: the population entering in direction q through a
// pressure face, from the one sent in direction inv_dir(q) (s_opp), the face
// density term rho (minus 1 in deviation units) and the cell's velocity u.
__device__ inline double abb_value(int q, double s_opp, double rho, const double u[3]) {
    double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return -s_opp + 2.0 * wq(q) * (rho + 4.5 * cu * cu - 1.5 * uu);
}

// Canonical f_q(x, t) of cell (x, y, z) from the stored (pulled) layout, in
// the units of S::to_f64 (the deviation for the deviation forms): the value
// streamed from x - c_q, or, through a face, the face rule applied to the
// population the cell sent against it (direction inv_dir(q)).
template <class S>
__device__ inline double pull_value(const BoxDev& bx, const typename S::T* g, int q, int x, int y, int z, float inv) {
    if (behind_side_wall(bx, x - CX[q], y - CY[q]))   // resting side wall: bounce-back
        return S::to_f64(g[pdf_index(bx, inv_dir(q), x, y, z)], inv);
    int zs = z - CZ[q];
    int w = face_of(bx, zs);
    if (w >= 0) {
        double so = S::to_f64(g[pdf_index(bx, inv_dir(q), x, y, z)], inv);
        if (bx.face_type[w] == FACE_PRESSURE) {
            double u[3];
            slot_velocity<S>(bx, g, x, y, z, inv, u);
            return abb_value(q, so, S::DEV ? bx.face_rho[w] - 1.0 : bx.face_rho[w], u);
        }
        return so + bx.bw[w][q];
    }
    int xs = x - CX[q], ys = y - CY[q];
    xs = xs < 0 ? xs + bx.nx : (xs >= bx.nx ? xs - bx.nx : xs);
    ys = ys < 0 ? ys + bx.ny : (ys >= bx.ny ? ys - bx.ny : ys);
    zs = zs < 0 ? zs + bx.nz : (zs >= bx.nz ? zs - bx.nz : zs);
    return S::to_f64(g[pdf_index(bx, q, xs, ys, zs)], inv);
}

// Inverse of pull_value for the 19 slots of cell (x, y, z): given the
// canonical field through canon(dir, cell) (FP64, full f), the slot values
// that pulling turns back into it. A slot whose reader is inside (or across
// a periodic boundary) holds the reader's value; a slot sent against a
// velocity face holds the cell's own opposite value minus the wall term; the
// slots sent against a pressure face solve the anti-bounce-back rule, whose
// velocity depends on all 19 slots, by fixed-point iteration (the
// dependence is quadratic in the velocity, so a few sweeps reach round-off).
template <class S, class Canon>
__device__ inline void store_cell_slots(const BoxDev& bx, typename S::T* g, int x, int y, int z, float scale,
                                        Canon canon) {
    const long long self = x + (long long)bx.nx * (y + (long long)bx.ny * z);
    double sl[NQ];
    int pface = -1;
    for (int q = 0; q < NQ; ++q) {
        int zd = z + CZ[q];
        int w = face_of(bx, zd);
        if (behind_side_wall(bx, x + CX[q], y + CY[q])) {
            sl[q] = canon(inv_dir(q), self);
        } else if (w < 0) {
            int xd = x + CX[q], yd = y + CY[q];
            xd = xd < 0 ? xd + bx.nx : (xd >= bx.nx ? xd - bx.nx : xd);
            yd = yd < 0 ? yd + bx.ny : (yd >= bx.ny ? yd - bx.ny : yd);
            zd = zd < 0 ? zd + bx.nz : (zd >= bx.nz ? zd - bx.nz : zd);
            sl[q] = canon(q, xd + (long long)bx.nx * (yd + (long long)bx.ny * zd));
        } else if (bx.face_type[w] == FACE_VELOCITY) {
            sl[q] = canon(inv_dir(q), self) - bx.bw[w][inv_dir(q)];
        } else {
            sl[q] = -canon(inv_dir(q), self) + 2.0 * wq(q) * bx.face_rho[w];
            pface = w;
        }
    }
    if (pface >= 0) {
        for (int it = 0; it < 12; ++it) {
            double u[3] = {0.0, 0.0, 0.0};
            for (int q = 1; q < NQ; ++q) {
                u[0] += sl[q] * CX[q]; u[1] += sl[q] * CY[q]; u[2] += sl[q] * CZ[q];
            }
            for (int q = 0; q < NQ; ++q)
                if (face_of(bx, z + CZ[q]) == pface && !behind_side_wall(bx, x + CX[q], y + CY[q]))
                    sl[q] = abb_value(q, canon(inv_dir(q), self), bx.face_rho[pface], u);
        }
    }
    for (int q = 0; q < NQ; ++q) {
        double v = S::DEV ? sl[q] - wq(q) : sl[q];
        g[pdf_index(bx, q, x, y, z)] = S::from_f64(v, scale);
    }
}

template <class S>
__global__ void k_set_pdfs(BoxDev bx, int parity, const double* __restrict__ f, float scale) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= bx.N) return;
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    typename S::T* g = (typename S::T*)bx.grid[parity];
    const long long N = bx.N;
    store_cell_slots<S>(bx, g, x, y, z, scale, [&](int d, long long c) { return f[(long long)d * N + c]; });
}

template <class S>
__global__ void k_set_equilibrium(BoxDev bx, int parity, const double* __restrict__ rho,
                                  const double* __restrict__ u, float scale) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= bx.N) return;
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    typename S::T* g = (typename S::T*)bx.grid[parity];
    const long long N = bx.N;
    // E_d(rho, u) of eq. (5) at cell c
    store_cell_slots<S>(bx, g, x, y, z, scale, [&](int d, long long c) {
        double r = rho ? rho[c] : 1.0;
        double vx = u[c], vy = u[N + c], vz = u[2 * N + c];
        double cv = CX[d] * vx + CY[d] * vy + CZ[d] * vz;
        double vv = vx * vx + vy * vy + vz * vz;
        return wq(d) * (r + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
    });
}

template <class S>
__global__ void k_get_pdfs(BoxDev bx, int parity, double* __restrict__ f, float inv) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= bx.N) return;
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    const typename S::T* g = (const typename S::T*)bx.grid[parity];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = pull_value<S>(bx, g, q, x, y, z, inv);
        if (S::DEV) v += wq(q);
        f[(long long)q * bx.N + n] = v;
    }
}

template <class S>
__global__ void k_get_pdfs_at(BoxDev bx, int parity, const int* __restrict__ cells, int ncells,
                              double* __restrict__ out, float inv, int* __restrict__ flags) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells) return;
    long long n = cells[i];
    if (n < 0 || n >= bx.N) {
        // an index outside the box reads nothing: NaN out, flag for the host
        for (int q = 0; q < NQ; ++q) out[(long long)q * ncells + i] = __builtin_nan("");
        atomicOr(flags, FLAG_BAD_CELL);
        return;
    }
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    const typename S::T* g = (const typename S::T*)bx.grid[parity];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = pull_value<S>(bx, g, q, x, y, z, inv);
        if (S::DEV) v += wq(q);
        out[(long long)q * ncells + i] = v;
    }
}

template <class S>
__global__ void k_macroscopic(BoxDev bx, int parity, double* __restrict__ rho, double* __restrict__ u,
                              float inv) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= bx.N) return;
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    const typename S::T* g = (const typename S::T*)bx.grid[parity];
    double r = 0, j[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double v = pull_value<S>(bx, g, q, x, y, z, inv);
        if (S::DEV) v += wq(q);
        r += v;
        j[0] += v * CX[q]; j[1] += v * CY[q]; j[2] += v * CZ[q];
    }
    rho[n] = r;
    u[n] = j[0] + 0.5 * bx.g[0];
    u[bx.N + n] = j[1] + 0.5 * bx.g[1];
    u[2LL * bx.N + n] = j[2] + 0.5 * bx.g[2];
}

// Dense two-slot solid fractions of one box (readout and overflow count),
// through the same candidate lists and mapping function as the step kernel.
__global__ void k_map_dense(BoxDev bx, Particles P, const int* __restrict__ tile_off,
                            const int* __restrict__ tile_pid, TileShape ts, double* __restrict__ B,
                            int* __restrict__ pid, unsigned long long* dropped) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= bx.N) return;
    int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
    int t = bx.tile_base + x / ts.tx + bx.ntx * (y / ts.ty + bx.nty * (z / ts.tz));
    int e0 = tile_off[t], e1 = tile_off[t + 1];
    Slots sl;
    slots_init(sl);
    for (int e = e0; e < e1; ++e) {
        int p = tile_pid[e];
        double dx = min_image((x + 0.5) - P.x[p], bx.L[0], bx.halfL[0]);
        double dy = min_image((y + 0.5) - P.y[p], bx.L[1], bx.halfL[1]);
        double dz = min_image((z + 0.5) - P.z[p], bx.L[2], bx.halfL[2]);
        double b = bx.mapping == 0 ? overlap_linear(dx, dy, dz, P.r[p], P.fr[p])
                                   : overlap_subsample(dx, dy, dz, P.r[p], bx.nsub, bx.sub_off, bx.reach);
        if (b > 0.0) slots_insert(sl, p, p, b);
    }
    slots_finish(sl);
    if (B) {
        B[n] = sl.c0 >= 0 ? sl.B0 : 0.0;
        B[bx.N + n] = sl.c1 >= 0 ? sl.B1 : 0.0;
    }
    if (pid) {
        pid[n] = sl.c0 >= 0 ? sl.c0 - bx.part_base : -1;
        pid[bx.N + n] = sl.c1 >= 0 ? sl.c1 - bx.part_base : -1;
    }
    if (sl.dropped) atomicAdd(dropped, (unsigned long long)sl.dropped);
}

// FP64 mass and momentum of the stored state (each slot is one f_q(x,t)):
// per-block partial sums, then one block adds them in a fixed order.
template <class S>
__global__ __launch_bounds__(256) void k_stats_partial(BoxDev bx, int parity, float inv, double* __restrict__ part) {
    __shared__ double s[4][256];
    const typename S::T* g = (const typename S::T*)bx.grid[parity];
    double m = 0, px = 0, py = 0, pz = 0;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < bx.N;
         n += (long long)gridDim.x * blockDim.x) {
        int x = n % bx.nx, y = (n / bx.nx) % bx.ny, z = n / ((long long)bx.nx * bx.ny);
        // each slot is one canonical value: the reader's f_q, or across a face
        // the cell's own f_opp(q) by the face rule
        double uc[3] = {0.0, 0.0, 0.0};
        const bool pz_face = bx.walls && ((z == 0 && bx.face_type[0] == FACE_PRESSURE) ||
                                          (z == bx.nz - 1 && bx.face_type[1] == FACE_PRESSURE));
        if (pz_face) slot_velocity<S>(bx, g, x, y, z, inv, uc);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double v = S::to_f64(g[pdf_index(bx, q, x, y, z)], inv);
            int d = q;
            int w = face_of(bx, z + CZ[q]);
            if (behind_side_wall(bx, x + CX[q], y + CY[q])) {
                d = inv_dir(q);
            } else if (w >= 0) {
                d = inv_dir(q);
                v = bx.face_type[w] == FACE_PRESSURE
                        ? abb_value(d, v, S::DEV ? bx.face_rho[w] - 1.0 : bx.face_rho[w], uc)
                        : v + bx.bw[w][d];
            }
            if (S::DEV) v += wq(q);
            m += v;
            px += v * CX[d]; py += v * CY[d]; pz += v * CZ[d];
        }
    }
    s[0][threadIdx.x] = m; s[1][threadIdx.x] = px; s[2][threadIdx.x] = py; s[3][threadIdx.x] = pz;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int k = 0; k < 4; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void k_stats_final(const double* part, int nblk, double* out) {
    if (threadIdx.x < 4) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += part[b * 4 + threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Plain streaming copy (bandwidth reference): one-shot grid, each thread
// moves one 16-byte vector (of the copy forms measured, the fastest).
__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ a, double2* __restrict__ b,
                                                     long long n) {
    long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Sphere integration (Sec. 2.2.2) for collision-free spheres, one thread per
// particle slot. m = rho_p (4/3) pi r^3, I = (2/5) m r^2; the total force is
// the hydrodynamic force of the last step plus m times the box's external
// acceleration, the torque is the hydrodynamic torque.
//   Euler:  x += dt U;  U += dt F/m;  Om += dt T/I.
//   Verlet (eqs. 15-16), once after each fluid step: complete the velocity
//   with the previous and the new force (skipped until a previous force
//   exists), then advance the position with the new one.
// Positions are wrapped into [0, L) along periodic axes; along an axis with
// walls a centre leaving [r + 1, L - r - 1] is mirrored back and its velocity
// component reversed (elastic contact keeping the mapping's one-cell gap).
// No fused multiply-add, so that the update is reproducible bit for bit.
template <int SCHEME>
__global__ __launch_bounds__(256) void k_integrate(IntParams ip) {
#pragma clang fp contract(off)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ip.P_total) return;
    const BoxDev& bx = ip.boxes[ip.part_box[p]];
    if (p - bx.part_base >= bx.np) return;
    const double pi = 3.14159265358979323846;
    const double dt = ip.dt, r = ip.P.r[p];
    const double m = bx.rho_p * (4.0 / 3.0) * pi * r * r * r;
    const double inertia = 0.4 * m * r * r;
    double* pos[3] = {ip.P.x, ip.P.y, ip.P.z};
    double* vel[3] = {ip.P.ux, ip.P.uy, ip.P.uz};
    double* ang[3] = {ip.P.ox, ip.P.oy, ip.P.oz};
    const double* acc = ip.P.acc + 6LL * p;
    double* fp = ip.P.fprev + 6LL * p;
    const bool prev = SCHEME == SCHEME_VERLET && ip.P.prev_ok[p] != 0;
    for (int a = 0; a < 3; ++a) {
        const double F = acc[a] + m * bx.accel[a];
        const double T = acc[3 + a];
        double x = pos[a][p], U = vel[a][p], W = ang[a][p];
        if (SCHEME == SCHEME_EULER) {
            x = x + dt * U;
            U = U + dt * F / m;
            W = W + dt * T / inertia;
        } else {
            if (prev) {
                U = U + dt / (2.0 * m) * (fp[a] + F);
                W = W + dt / (2.0 * inertia) * (fp[3 + a] + T);
            }
            x = x + (dt * U + dt * dt / (2.0 * m) * F);
            fp[a] = F;
            fp[3 + a] = T;
        }
        const double L = bx.L[a];
        const bool walled = a == 2 ? bx.walls != 0 : (bx.walls_xy & (1 << a)) != 0;
        if (walled) {
            // elastic contact one cell before the walls: mirror the centre back
            // into [r + 1, L - r - 1] and reverse the normal velocity
            const double lo = r + 1.0, hi = L - r - 1.0;
            if (x < lo) { x = 2.0 * lo - x; U = -U; }
            else if (x > hi) { x = 2.0 * hi - x; U = -U; }
        } else {
            double w = x - L * floor(x / L);
            if (w >= L) w -= L;
            if (w < 0.0) w = 0.0;
            x = w;
        }
        pos[a][p] = x;
        vel[a][p] = U;
        ang[a][p] = W;
    }
    if (SCHEME == SCHEME_VERLET) ip.P.prev_ok[p] = 1;
}

// Replace the list bits of the error word by those of the lists just built
// (report = 0: clear them only, for a build whose counts the host checks).
__global__ void k_check_lists(const int* __restrict__ stats, long long cap, int* __restrict__ err, int report) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int e = 0;
        if ((long long)stats[1] > cap) e |= FLAG_LIST_ENTRIES;
        if (stats[0] > MAXC) e |= FLAG_LIST_TILE;
        err[0] = (err[0] & ~(FLAG_LIST_ENTRIES | FLAG_LIST_TILE)) | (report ? e : 0);
    }
}

// ---------------------------------------------------------------------------
// FP64 totals of a canonical field without a context or a workspace, for
// callers that cannot allocate device memory. The per-block partial sums go
// to a library-owned array (one copy per GPU, alive until the process ends):
// block b sums cells [b * NOALLOC_CELLS_PER_BLOCK, (b + 1) * ...), each
// thread 64 cells 256 apart in cell order, then a fixed tree in LDS; one
// more kernel adds the blocks in order. Every partial slot a call reads was
// written by the same call, so nothing needs clearing; calls that overlap on
// one GPU (different streams) race on the array.
constexpr int NOALLOC_BLOCKS = 4096;
constexpr long long NOALLOC_CELLS_PER_BLOCK = 256LL * 64;
static __device__ __align__(256) double scratch[NOALLOC_BLOCKS * 4];

__global__ __launch_bounds__(256) void k_field_stats_partial(const double* __restrict__ f, long long N,
                                                             double* __restrict__ part) {
    __shared__ double s[4][256];
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    const long long c0 = (long long)blockIdx.x * NOALLOC_CELLS_PER_BLOCK + threadIdx.x;
    for (int k = 0; k < 64; ++k) {
        const long long n = c0 + 256LL * k;
        if (n >= N) break;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double v = f[(long long)q * N + n];
            m += v;
            px += v * CX[q]; py += v * CY[q]; pz += v * CZ[q];
        }
    }
    s[0][threadIdx.x] = m; s[1][threadIdx.x] = px; s[2][threadIdx.x] = py; s[3][threadIdx.x] = pz;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int k = 0; k < 4; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

// Device address of `scratch` on each GPU, looked up once per device with
// that device current (the array's name is only a host-side stand-in).
static double* g_scratch_dev[64];
static std::mutex g_scratch_mu;

static hipError_t scratch_of_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = (double*)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

long long noalloc_max_cells() { return NOALLOC_BLOCKS * NOALLOC_CELLS_PER_BLOCK; }

hipError_t launch_field_stats_noalloc(const double* f, long long N, double* out, hipStream_t st) {
    double* part = nullptr;
    hipError_t e = scratch_of_current_device(&part);
    if (e != hipSuccess) return e;
    const int nblk = (int)((N + NOALLOC_CELLS_PER_BLOCK - 1) / NOALLOC_CELLS_PER_BLOCK);
    if (nblk > NOALLOC_BLOCKS) return hipErrorInvalidValue;
    if (nblk > 0) hipLaunchKernelGGL(k_field_stats_partial, dim3(nblk), dim3(256), 0, st, f, N, part);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nblk, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers (called by the engine).

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// The step kernel instance for (storage, map, filt): storage psm_storage;
// map 0 when every box uses the linear approximation, 1 if any box samples;
// filt the per-wave candidate filter.
// ---------------------------------------------------------------------------
// Bandwidth reference for the step's access pattern: the tile walk, pulls and
// stores of k_psm_step with no arithmetic. SHIFT pulls each direction from
// x - c_q on the source planes z, z -+ 1 as the step does; otherwise every
// direction comes from the cell itself. Values are stored unchanged at the
// cell in the other grid (the source grid is not written).
template <class S, bool SHIFT>
__global__ __launch_bounds__(WG) void k_pattern_copy(StepParams kp) {
    using R = typename S::R;
    using T = typename S::T;
    const int tid = threadIdx.x;
    const int TX = kp.tx, TY = kp.ty, TZ = kp.tz;
    const int lx = tid % TX, ly = tid / TX;
    const int G = gridDim.x;
    const int xcd = blockIdx.x % NXCD;
    const int gx8 = (G - xcd + NXCD - 1) / NXCD;
    const int t_begin = (int)(((long long)kp.T_total * xcd) / NXCD);
    const int t_end = (int)(((long long)kp.T_total * (xcd + 1)) / NXCD);
    const PSM_CONST BoxDev* boxes = cptr(kp.boxes);
    for (int t = t_begin + (int)blockIdx.x / NXCD; t < t_end; t += gx8) {
        int b = 0;
        if (kp.nbox > 1) {
            const PSM_CONST int* tb = cptr(kp.box_tile_base);
            int lo = 0, hi = kp.nbox - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (tb[mid] <= t) lo = mid; else hi = mid - 1;
            }
            b = lo;
        }
        const PSM_CONST BoxDev& bx = boxes[b];
        const int nx = bx.nx, ny = bx.ny, nz = bx.nz;
        const int lt = t - bx.tile_base;
        const int tcx = lt % bx.ntx, tcy = (lt / bx.ntx) % bx.nty, tcz = lt / (bx.ntx * bx.nty);
        const int x = tcx * TX + lx, y = tcy * TY + ly;
        if (x >= nx || y >= ny) continue;
        const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
        const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
        const int pitch = bx.pitch;
        auto inplane = [pitch](int xx, int yy) -> unsigned {
            int c = xx + pitch * yy;
            return (unsigned)(((c / BLK) * (NQ * BLK) + (c % BLK)) * (int)sizeof(T));
        };
        const unsigned o00 = inplane(x, y);
        const unsigned om0 = SHIFT ? inplane(xm, y) : o00, op0 = SHIFT ? inplane(xp, y) : o00;
        const unsigned o0m = SHIFT ? inplane(x, ym) : o00, o0p = SHIFT ? inplane(x, yp) : o00;
        const unsigned omm = SHIFT ? inplane(xm, ym) : o00, opp = SHIFT ? inplane(xp, yp) : o00;
        const unsigned omp = SHIFT ? inplane(xm, yp) : o00, opm = SHIFT ? inplane(xp, ym) : o00;
        const long long pbytes = bx.plane_elems * (long long)sizeof(T);
        const unsigned pb32 = (unsigned)pbytes;
        const char* src = (const char*)bx.grid[kp.parity];
        const char* dst = (const char*)bx.grid[kp.parity ^ 1];
        constexpr int QB = BLK * (int)sizeof(T);
        for (int k = 0; k < TZ; ++k) {
            const int z = tcz * TZ + k;
            if (z >= nz) break;
            const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
            const Rsrc sz = plane_rsrc(src + z * pbytes, pb32);
            const Rsrc sm = SHIFT ? plane_rsrc(src + zm * pbytes, pb32) : sz;
            const Rsrc sp = SHIFT ? plane_rsrc(src + zp * pbytes, pb32) : sz;
            const Rsrc dz_ = plane_rsrc(dst + z * pbytes, pb32);
            R f[NQ];
            PSM_LOAD19(f, sz, sm, sp);
#pragma unroll
            for (int q = 0; q < NQ; ++q) S::st(dz_, o00, q * QB, f[q]);
        }
    }
}

hipError_t launch_pattern_copy(int storage, bool shifted, const StepParams& kp, int grid, hipStream_t st) {
    const void* k;
    switch (storage) {
        case 0: k = shifted ? (const void*)k_pattern_copy<St64, true> : (const void*)k_pattern_copy<St64, false>; break;
        case 1: k = shifted ? (const void*)k_pattern_copy<St32, true> : (const void*)k_pattern_copy<St32, false>; break;
        default: k = shifted ? (const void*)k_pattern_copy<St16, true> : (const void*)k_pattern_copy<St16, false>;
    }
    void* args[] = {(void*)&kp};
    return hipLaunchKernel(k, dim3(grid), dim3(WG), args, 0, st);
}

template <int MAP, bool FILT>
static const void* step_kernel_of(int storage) {
    switch (storage) {
        case 0: return (const void*)k_psm_step<St64, MAP, FILT>;
        case 1: return (const void*)k_psm_step<St32, MAP, FILT>;
        default: return (const void*)k_psm_step<St16, MAP, FILT>;
    }
}

static const void* step_kernel(int storage, int map, bool filt) {
    if (map) return filt ? step_kernel_of<1, true>(storage) : step_kernel_of<1, false>(storage);
    return filt ? step_kernel_of<0, true>(storage) : step_kernel_of<0, false>(storage);
}

hipError_t launch_step(int storage, int map, bool filt, const StepParams& kp, int grid, hipStream_t st) {
    void* args[] = {(void*)&kp};
    return hipLaunchKernel(step_kernel(storage, map, filt), dim3(grid), dim3(WG), args, 0, st);
}

int step_blocks_per_cu(int storage, int map, bool filt) {
    int nb = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel(storage, map, filt), WG, 0);
    return nb > 0 ? nb : 1;
}

hipError_t launch_reduce(const ReduceParams& rp, hipStream_t st) {
    if (rp.P_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_forces, dim3(blocks_for(rp.P_total, 4)), dim3(256), 0, st, rp);
    return hipGetLastError();
}

int scan_chunks(int n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK; }

// scratch: 2 * scan_chunks(T) ints
hipError_t launch_bin(const BinParams& bp, int* stats, int* scratch, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(bp.T_total, 256) > 4096 ? 4096 : blocks_for(bp.T_total, 256)),
                       dim3(256), 0, st, bp.tile_cnt, (long long)bp.T_total, 0);
    if (bp.P_total > 0)
        hipLaunchKernelGGL(k_bin<false>, dim3(blocks_for(bp.P_total, 4)), dim3(256), 0, st, bp);
    int nch = scan_chunks(bp.T_total);
    int* csum = scratch;
    int* cmax = scratch + nch;
    hipLaunchKernelGGL(k_scan_chunks, dim3(nch), dim3(256), 0, st, bp.tile_cnt, bp.T_total, csum, cmax);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, st, csum, cmax, nch, stats);
    hipLaunchKernelGGL(k_scan_apply, dim3(nch), dim3(256), 0, st, bp.tile_cnt, bp.T_total, csum, bp.tile_off,
                       stats);
    return hipGetLastError();
}

hipError_t launch_bin_fill(const BinParams& bp, hipStream_t st) {
    if (bp.P_total > 0)
        hipLaunchKernelGGL(k_bin<true>, dim3(blocks_for(bp.P_total, 4)), dim3(256), 0, st, bp);
    return hipGetLastError();
}

hipError_t launch_set_pdfs(int storage, const BoxDev& bx, int parity, const double* f, float scale,
                           hipStream_t st) {
    unsigned g = blocks_for(bx.N, 256);
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_set_pdfs<St64>, dim3(g), dim3(256), 0, st, bx, parity, f, scale); break;
        case 1: hipLaunchKernelGGL(k_set_pdfs<St32>, dim3(g), dim3(256), 0, st, bx, parity, f, scale); break;
        default: hipLaunchKernelGGL(k_set_pdfs<St16>, dim3(g), dim3(256), 0, st, bx, parity, f, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_set_equilibrium(int storage, const BoxDev& bx, int parity, const double* rho, const double* u,
                                  float scale, hipStream_t st) {
    unsigned g = blocks_for(bx.N, 256);
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_set_equilibrium<St64>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, scale); break;
        case 1: hipLaunchKernelGGL(k_set_equilibrium<St32>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, scale); break;
        default: hipLaunchKernelGGL(k_set_equilibrium<St16>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, scale); break;
    }
    return hipGetLastError();
}

hipError_t launch_get_pdfs(int storage, const BoxDev& bx, int parity, double* f, float inv, hipStream_t st) {
    unsigned g = blocks_for(bx.N, 256);
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_get_pdfs<St64>, dim3(g), dim3(256), 0, st, bx, parity, f, inv); break;
        case 1: hipLaunchKernelGGL(k_get_pdfs<St32>, dim3(g), dim3(256), 0, st, bx, parity, f, inv); break;
        default: hipLaunchKernelGGL(k_get_pdfs<St16>, dim3(g), dim3(256), 0, st, bx, parity, f, inv); break;
    }
    return hipGetLastError();
}

hipError_t launch_get_pdfs_at(int storage, const BoxDev& bx, int parity, const int* cells, int ncells, double* out,
                              float inv, int* flags, hipStream_t st) {
    unsigned g = blocks_for(ncells, 256);
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_get_pdfs_at<St64>, dim3(g), dim3(256), 0, st, bx, parity, cells, ncells, out, inv, flags); break;
        case 1: hipLaunchKernelGGL(k_get_pdfs_at<St32>, dim3(g), dim3(256), 0, st, bx, parity, cells, ncells, out, inv, flags); break;
        default: hipLaunchKernelGGL(k_get_pdfs_at<St16>, dim3(g), dim3(256), 0, st, bx, parity, cells, ncells, out, inv, flags); break;
    }
    return hipGetLastError();
}

hipError_t launch_macroscopic(int storage, const BoxDev& bx, int parity, double* rho, double* u, float inv,
                              hipStream_t st) {
    unsigned g = blocks_for(bx.N, 256);
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_macroscopic<St64>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, inv); break;
        case 1: hipLaunchKernelGGL(k_macroscopic<St32>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, inv); break;
        default: hipLaunchKernelGGL(k_macroscopic<St16>, dim3(g), dim3(256), 0, st, bx, parity, rho, u, inv); break;
    }
    return hipGetLastError();
}

hipError_t launch_map_dense(const BoxDev& bx, const Particles& P, const int* tile_off, const int* tile_pid,
                            TileShape ts, double* B, int* pid, unsigned long long* dropped, hipStream_t st) {
    hipLaunchKernelGGL(k_map_dense, dim3(blocks_for(bx.N, 256)), dim3(256), 0, st, bx, P, tile_off, tile_pid, ts,
                       B, pid, dropped);
    return hipGetLastError();
}

int stats_blocks() { return 1024; }

hipError_t launch_stats(int storage, const BoxDev& bx, int parity, float inv, double* part, double* out,
                        hipStream_t st) {
    int nb = stats_blocks();
    switch (storage) {
        case 0: hipLaunchKernelGGL(k_stats_partial<St64>, dim3(nb), dim3(256), 0, st, bx, parity, inv, part); break;
        case 1: hipLaunchKernelGGL(k_stats_partial<St32>, dim3(nb), dim3(256), 0, st, bx, parity, inv, part); break;
        default: hipLaunchKernelGGL(k_stats_partial<St16>, dim3(nb), dim3(256), 0, st, bx, parity, inv, part); break;
    }
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_integrate(int scheme, const IntParams& ip, hipStream_t st) {
    if (ip.P_total == 0) return hipSuccess;
    if (scheme == SCHEME_EULER)
        hipLaunchKernelGGL(k_integrate<SCHEME_EULER>, dim3(blocks_for(ip.P_total, 256)), dim3(256), 0, st, ip);
    else
        hipLaunchKernelGGL(k_integrate<SCHEME_VERLET>, dim3(blocks_for(ip.P_total, 256)), dim3(256), 0, st, ip);
    return hipGetLastError();
}

hipError_t launch_check_lists(const int* stats, long long cap, int* err, int report, hipStream_t st) {
    hipLaunchKernelGGL(k_check_lists, dim3(1), dim3(64), 0, st, stats, cap, err, report);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* a, long long n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    unsigned nb = blocks_for(n, 256);
    hipLaunchKernelGGL(k_fill_int, dim3(nb > 4096 ? 4096 : nb), dim3(256), 0, st, a, n, v);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
    long long n = (long long)(bytes / 16);
    long long blocks = (n + 255) / 256;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, (const double2*)src, (double2*)dst,
                       n);
    return hipGetLastError();
}

}  // namespace psm
