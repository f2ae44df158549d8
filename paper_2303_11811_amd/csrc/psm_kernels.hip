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

#define GLOBAL __attribute__((address_space(1)))
typedef const GLOBAL char GCHAR;

// Cache policy of the PDF streams (compile-time switches, measured by the
// autotuning sweeps): nontemporal stores / loads bypass cache retention.
#ifndef PSM_NT_STORE
#define PSM_NT_STORE 1
#endif
#ifndef PSM_NT_LOAD
#define PSM_NT_LOAD 0
#endif
template <class T> __device__ __forceinline__ T ld_pdf(const GLOBAL T* p) {
#if PSM_NT_LOAD
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <class T> __device__ __forceinline__ void st_pdf(GLOBAL T* p, T v) {
#if PSM_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

// ---------------------------------------------------------------------------
// Storage traits: FP64 stores f; the deviation forms store d = f - w_q
// (FP16 as scale * d) and compute in FP32.
struct St64 {
    using T = double;
    using R = double;
    static constexpr bool DEV = false;
    static constexpr bool SCALED = false;
    __device__ static R loadb(const GCHAR* b, unsigned off, float) { return ld_pdf((const GLOBAL T*)(b + off)); }
    __device__ static void storeb(GLOBAL char* b, unsigned off, R v, float) { st_pdf((GLOBAL T*)(b + off), v); }
    __device__ static double to_f64(T v, float) { return v; }
    __device__ static T from_f64(double v, float) { return v; }
};
struct St32 {
    using T = float;
    using R = float;
    static constexpr bool DEV = true;
    static constexpr bool SCALED = false;
    __device__ static R loadb(const GCHAR* b, unsigned off, float) { return ld_pdf((const GLOBAL T*)(b + off)); }
    __device__ static void storeb(GLOBAL char* b, unsigned off, R v, float) { st_pdf((GLOBAL T*)(b + off), v); }
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
    __device__ static R loadb(const GCHAR* b, unsigned off, float) { return (float)ld_pdf((const GLOBAL T*)(b + off)); }
    __device__ static void storeb(GLOBAL char* b, unsigned off, R v, float) { st_pdf((GLOBAL T*)(b + off), (_Float16)v); }
    // scale is a power of two: multiplication by it and by 1/scale is exact
    __device__ static double to_f64(T v, float inv) { return (double)((float)v * inv); }
    __device__ static T from_f64(double v, float scale) { return (_Float16)(float)(v * (double)scale); }
};

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

// Cross-lane moves of a double. DPP forms stay inside a row of 16 lanes and
// run on the vector ALU: quad permutations, the mirror inside each half row
// (lane i <-> 7 - i of its group of 8) and the rotation of a row by 8 (lane
// i <-> i ^ 8). Lane i ^ 16 comes from a swizzle inside 32 lanes, lane i ^ 32
// from a permute.
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
__device__ __forceinline__ double swizzle_xor16(double v) {
    // bit mode: and mask 0x1f, or mask 0, xor mask 0x10
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)b, 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Wave sums of six values at once. Inside each group of 8 lanes a butterfly
// splits the values (padded to 8) between exchanging lanes: the mirror pair
// by bit 2 of the lane, then quad partners by bits 1 and 0 (7 exchanges),
// after which lane l holds the group's sum of value l & 7; three exchanges
// across groups finish the sums. All within-group moves are DPP. Every lane
// returns the total of value `comp` = l & 7 (values 6 and 7 are padding).
// The order of the additions is fixed, so the result is reproducible bit for
// bit, and partners add the same two numbers, so all lanes of one value agree.
__device__ inline double wave_sum6(const double v[6], int lane, int& comp) {
    const bool b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
    double a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double lo = v[i], hi = i + 4 < 6 ? v[i + 4] : 0.0;
        const double keep = b2 ? hi : lo, send = b2 ? lo : hi;
        a[i] = keep + dpp_f64<DPP_ROW_HALF_MIRROR>(send);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = b1 ? a[i + 2] : a[i], send = b1 ? a[i] : a[i + 2];
        b[i] = keep + dpp_f64<DPP_QUAD_XOR2>(send);
    }
    const double keep = b0 ? b[1] : b[0], send = b0 ? b[0] : b[1];
    double d = keep + dpp_f64<DPP_QUAD_XOR1>(send);
    d += dpp_f64<DPP_ROW_ROR8>(d);
    d += swizzle_xor16(d);
    d += __shfl_xor(d, 32, 64);
    comp = lane & 7;
    return d;
}

// Uniform (wave-invariant) data is read through the constant address space so
// that it lands in scalar registers.
#define PSM_CONST __attribute__((address_space(4)))
template <class T> __device__ __forceinline__ const PSM_CONST T* cptr(const T* p) {
    return (const PSM_CONST T*)p;
}

// One inverse pair (q, q+1) of the plain SRT update with forcing:
//   E_q(U) = w (rho + 3 c.U + 4.5 (c.U)^2 - 1.5 U.U) = s + a, E_qbar(U) = s - a  (eq. 5)
//   t_q = (E_q(U) - f_q)/tau + F_q      (eq. 3; eq. 8 with the Guo prefactor)
//   f~_q = f_q + t_q
// rho is the density deviation for the deviation storage forms.
template <class R, int Q>
__device__ __forceinline__ void pair_fluid(R& fq, R& fb, R base, R Ux, R Uy, R Uz, R fa, R fs, R pwUg3,
                                           R omega, R k45) {
    constexpr R w = (R)wq(Q);
    constexpr R cx = (R)CX[Q], cy = (R)CY[Q], cz = (R)CZ[Q];
    R cu = cx * Ux + cy * Uy + cz * Uz;
    R sU = w * base + (k45 * w) * (cu * cu);
    R aU = ((R)3.0 * w) * cu;
    R Fs = fs * cu - pwUg3;
    fq = fq + (omega * (sU + aU - fq) + (Fs + fa));
    fb = fb + (omega * (sU - aU - fb) + (Fs - fa));
}

// The same pair under PSM (eqs. 17-19):
//   f~_q = f_q + (1-B) t_q + B (f_qbar - E_qbar(U) - f_q) + sum_s B_s E_q(U_p,s)
// with the slot sum folded into ten cell scalars:
//   sum_s B_s E_q(V_s) = w (A0 + 4.5 c.M.c) + 3 w c.P,
//   A0 = sum_s B_s (rho - 1.5 V_s.V_s), M = sum_s B_s V_s V_s^T, P = sum_s B_s V_s.
template <class R, int Q>
__device__ __forceinline__ void pair_psm(R& fq, R& fb, R base, R Ux, R Uy, R Uz, R fa, R fs, R pwUg3, R omega,
                                         R k45, R Bt, R omB, R A0, R Mxx, R Myy, R Mzz, R Mxy, R Mxz, R Myz,
                                         R Px, R Py, R Pz) {
    constexpr R w = (R)wq(Q);
    constexpr int ix = CX[Q], iy = CY[Q], iz = CZ[Q];
    constexpr R cx = (R)ix, cy = (R)iy, cz = (R)iz;
    R cu = cx * Ux + cy * Uy + cz * Uz;
    R sU = w * base + (k45 * w) * (cu * cu);
    R aU = ((R)3.0 * w) * cu;
    R Fs = fs * cu - pwUg3;
    R tq = omega * (sU + aU - fq) + (Fs + fa);
    R tb = omega * (sU - aU - fb) + (Fs - fa);
    R cMc = (R)(ix * ix) * Mxx + (R)(iy * iy) * Myy + (R)(iz * iz) * Mzz +
            (R)(2 * ix * iy) * Mxy + (R)(2 * ix * iz) * Mxz + (R)(2 * iy * iz) * Myz;
    R cP = cx * Px + cy * Py + cz * Pz;
    R sV = w * A0 + (k45 * w) * cMc;
    R aV = ((R)3.0 * w) * cP;
    R Sq = Bt * (fb - (sU - aU) - fq) + (sV + aV);
    R Sb = Bt * (fq - (sU + aU) - fb) + (sV - aV);
    R nq = (fq + omB * tq) + Sq;
    R nb = (fb + omB * tb) + Sb;
    fq = nq;
    fb = nb;
}

// Lever arm d = x - x_p (minimum image, taken in FP64) and particle velocity
// at the cell centre (eq. 20) times the storage scale sc, in the collision's
// precision R: FP64 for FP64 storage, FP32 for the deviation forms.
template <class R>
__device__ __forceinline__ void slot_geometry(int c, double cxc, double cyc, double czc, double Lx, double hLx,
                                              double Ly, double hLy, double Lz, double hLz, const double* px,
                                              const double* py, const double* pz, const double* ux,
                                              const double* uy, const double* uz, const double* ox,
                                              const double* oy, const double* oz, R sc, R& dx, R& dy, R& dz,
                                              R& Vx, R& Vy, R& Vz) {
    dx = (R)min_image(cxc - px[c], Lx, hLx);
    dy = (R)min_image(cyc - py[c], Ly, hLy);
    dz = (R)min_image(czc - pz[c], Lz, hLz);
    Vx = sc * ((R)ux[c] + ((R)oy[c] * dz - (R)oz[c] * dy));
    Vy = sc * ((R)uy[c] + ((R)oz[c] * dx - (R)ox[c] * dz));
    Vz = sc * ((R)uz[c] + ((R)ox[c] * dy - (R)oy[c] * dx));
}

// Waves per SIMD the register budget of the step kernel is cut for: 3 for
// FP64 and FP16 storage (168 VGPRs), 4 for FP32 storage (128 VGPRs). Under
// the 128-register cap the FP16 form serialises its 19 loads.
#ifndef PSM_WAVES_PER_EU
#define PSM_WAVES_PER_EU 3
#endif
#ifndef PSM_WAVES_PER_EU_F32
#define PSM_WAVES_PER_EU_F32 4
#endif

// pull of the 19 values of one cell: planes z (bz), z-1 (bm), z+1 (bp)
#define PSM_LOAD19(F, bz, bm, bp)                      \
    do {                                               \
        F[0] = S::loadb(bz + 0 * QB, o00, kp.h_inv);   \
        F[1] = S::loadb(bz + 1 * QB, om0, kp.h_inv);   \
        F[2] = S::loadb(bz + 2 * QB, op0, kp.h_inv);   \
        F[3] = S::loadb(bz + 3 * QB, o0m, kp.h_inv);   \
        F[4] = S::loadb(bz + 4 * QB, o0p, kp.h_inv);   \
        F[5] = S::loadb(bm + 5 * QB, o00, kp.h_inv);   \
        F[6] = S::loadb(bp + 6 * QB, o00, kp.h_inv);   \
        F[7] = S::loadb(bz + 7 * QB, omm, kp.h_inv);   \
        F[8] = S::loadb(bz + 8 * QB, opp, kp.h_inv);   \
        F[9] = S::loadb(bz + 9 * QB, omp, kp.h_inv);   \
        F[10] = S::loadb(bz + 10 * QB, opm, kp.h_inv); \
        F[11] = S::loadb(bm + 11 * QB, om0, kp.h_inv); \
        F[12] = S::loadb(bp + 12 * QB, op0, kp.h_inv); \
        F[13] = S::loadb(bp + 13 * QB, om0, kp.h_inv); \
        F[14] = S::loadb(bm + 14 * QB, op0, kp.h_inv); \
        F[15] = S::loadb(bm + 15 * QB, o0m, kp.h_inv); \
        F[16] = S::loadb(bp + 16 * QB, o0p, kp.h_inv); \
        F[17] = S::loadb(bp + 17 * QB, o0m, kp.h_inv); \
        F[18] = S::loadb(bm + 18 * QB, o0p, kp.h_inv); \
    } while (0)
template <class S, int MAP, bool FILT>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(sizeof(typename S::T) == 4 ? PSM_WAVES_PER_EU_F32 : PSM_WAVES_PER_EU, 8))) void k_psm_step(
    StepParams kp) {
    using R = typename S::R;
    using T = typename S::T;

    __shared__ double s_px[MAXC], s_py[MAXC], s_pz[MAXC], s_pr[MAXC], s_pfr[MAXC];
    __shared__ double s_ux[MAXC], s_uy[MAXC], s_uz[MAXC], s_ox[MAXC], s_oy[MAXC], s_oz[MAXC];
    __shared__ int s_pid[MAXC];
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

    for (int t = t_begin + m; t < t_end; t += gx8) {
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

        if (nc > 0) {
            for (int c = tid; c < nc; c += WG) {
                int p = kp.tile_pid[e0 + c];
                s_pid[c] = p;
                s_px[c] = kp.P.x[p]; s_py[c] = kp.P.y[p]; s_pz[c] = kp.P.z[p];
                s_pr[c] = kp.P.r[p]; s_pfr[c] = kp.P.fr[p];
                s_ux[c] = kp.P.ux[p]; s_uy[c] = kp.P.uy[p]; s_uz[c] = kp.P.uz[p];
                s_ox[c] = kp.P.ox[p]; s_oy[c] = kp.P.oy[p]; s_oz[c] = kp.P.oz[p];
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
        // they do not depend on z
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
        const T* __restrict__ src = (const T*)bx.grid[kp.parity];
        T* __restrict__ dst = (T*)bx.grid[kp.parity ^ 1];
        const R omega = (R)bx.omega;
        const R gx = (R)bx.g[0], gy = (R)bx.g[1], gz = (R)bx.g[2];
        // scaled storage (FP16): the kernel works on s d; the quadratic terms
        // carry 1/s and every particle velocity is multiplied by s
        const R sc = S::SCALED ? (R)kp.h_scale : (R)1;
        const R k15 = S::SCALED ? (R)1.5 * (R)kp.h_inv : (R)1.5;
        const R k45 = S::SCALED ? (R)4.5 * (R)kp.h_inv : (R)4.5;
        const double Lx = bx.L[0], Ly = bx.L[1], Lz = bx.L[2];
        const double hLx = bx.halfL[0], hLy = bx.halfL[1], hLz = bx.halfL[2];
        const double cxc = xs + 0.5, cyc = ys + 0.5;
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

        for (int k = 0; k < TZ; ++k) {
            const int z = tcz * TZ + k;
            if (z >= nz) break;
            const double czc = z + 0.5;
            const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
            // scalar plane bases of the source planes z-1, z, z+1 and the
            // destination plane z; directions are 64 values apart in a block
            const GCHAR* sbz = (const GCHAR*)src + z * pbytes;
            const GCHAR* sbm = (const GCHAR*)src + zm * pbytes;
            const GCHAR* sbp = (const GCHAR*)src + zp * pbytes;
            GLOBAL char* dbz = (GLOBAL char*)dst + z * pbytes;

            // 1. solid fractions of this cell from the staged candidates (Sec. 2.3.2);
            // with the filter, only the candidates that can reach this wave at this z
            int c0 = -1, c1 = -1;
            double B0 = 0.0, B1 = 0.0;
            int dropped = 0;   // overlaps beyond the two slots at this cell
#define PSM_MAP_ONE(c)                                                                                       \
    do {                                                                                                    \
        double dx = min_image(cxc - s_px[c], Lx, hLx);                                                      \
        double dy = min_image(cyc - s_py[c], Ly, hLy);                                                      \
        double dz = min_image(czc - s_pz[c], Lz, hLz);                                                      \
        double B = lin_map ? overlap_linear(dx, dy, dz, s_pr[c], s_pfr[c])                                  \
                            : overlap_subsample(dx, dy, dz, s_pr[c], bx.nsub, bx.sub_off, bx.reach);         \
        if (B > 0.0) slots_insert(sl, c, s_pid[c], B);                                                      \
    } while (0)
            if constexpr (FILT) {
                unsigned long long cm = nc > 0 ? s_cmask[wave][k] : 0ull;
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

            // 2. pull: f_q(x) = grid[q][x - c_q]
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
                            fb[i] = S::loadb(sbz + inv_dir(q) * QB, o00, kp.h_inv) + ws * (R)bx.bw[w][q];
                        }
                    } else {
                        // anti-bounce-back with the cell's post-collision velocity
                        // (its own 19 slots); deviation units carry rho_w - 1
                        R ux = 0, uy = 0, uz = 0;
#pragma unroll
                        for (int q = 1; q < NQ; ++q) {
                            const R v = S::loadb(sbz + q * QB, o00, kp.h_inv);
                            ux += (R)CX[q] * v; uy += (R)CY[q] * v; uz += (R)CZ[q] * v;
                        }
                        const R rw = S::DEV ? (R)(bx.face_rho[w] - 1.0) * sc : (R)bx.face_rho[w];
                        const R uu = k15 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
                        for (int i = 0; i < 5; ++i) {
                            const int q = w == 0 ? in0[i] : in1[i];
                            const R cu = (R)CX[q] * ux + (R)CY[q] * uy + (R)CZ[q] * uz;
                            fb[i] = (R)(2.0 * wq(q)) * (rw + k45 * (cu * cu) - uu) -
                                    S::loadb(sbz + inv_dir(q) * QB, o00, kp.h_inv);
                        }
                    }
                }
                R f[NQ];
                PSM_LOAD19(f, sbz, sbm, sbp);
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
                        if (hit) f[q] = S::loadb(sbz + inv_dir(q) * QB, o00, kp.h_inv);
                    }
                }

                // 3. moments, eqs. (6)-(7); U carries the f/2 shift
                R rho = ((((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) +
                         (((f[8] + f[9]) + (f[10] + f[11])) + ((f[12] + f[13]) + (f[14] + f[15])))) +
                        ((f[16] + f[17]) + f[18]);
                R jx = ((f[1] - f[2]) + (f[7] - f[8])) + ((f[9] - f[10]) + (f[11] - f[12])) + (f[13] - f[14]);
                R jy = ((f[3] - f[4]) + (f[7] - f[8])) + ((f[10] - f[9]) + (f[15] - f[16])) + (f[17] - f[18]);
                R jz = ((f[5] - f[6]) + (f[11] - f[12])) + ((f[14] - f[13]) + (f[15] - f[16])) + (f[18] - f[17]);
                const R half = (R)0.5;
                R Ux = jx + half * (sc * gx), Uy = jy + half * (sc * gy), Uz = jz + half * (sc * gz);
                R uu = Ux * Ux + Uy * Uy + Uz * Uz;
                R base = rho - k15 * uu;
                R Ug3 = (R)3.0 * (Ux * gx + Uy * gy + Uz * gz);
                const R pu0 = (R)bx.pw[0] * Ug3, pu1 = (R)bx.pw[1] * Ug3, pu2 = (R)bx.pw[2] * Ug3;

                // 4. collision; each pair is stored as soon as it is final
#define PSM_STORE(Q) S::storeb(dbz + (Q) * QB, o00, f[Q], kp.h_scale)
                if (!psm_wave) {
                    f[0] = f[0] + (omega * ((R)W0 * base - f[0]) - pu0);
                    PSM_STORE(0);
#define PSM_PAIR(Q)                                                                                           \
    pair_fluid<R, Q>(f[Q], f[Q + 1], base, Ux, Uy, Uz, (R)(S::SCALED ? bx.fa_scaled[Q / 2] : bx.fa[Q / 2]),  \
                     (R)bx.fs[Q / 2], Q < 7 ? pu1 : pu2, omega, k45);                                         \
    PSM_STORE(Q);                                                                                             \
    PSM_STORE(Q + 1)
                    PSM_PAIR(1); PSM_PAIR(3); PSM_PAIR(5); PSM_PAIR(7); PSM_PAIR(9);
                    PSM_PAIR(11); PSM_PAIR(13); PSM_PAIR(15); PSM_PAIR(17);
#undef PSM_PAIR
                } else {
                    hx = (R)2 * jx - Ux; hy = (R)2 * jy - Uy; hz = (R)2 * jz - Uz;
                    // slot terms with U_p(x) of eq. (20)
                    R Bt = 0, A0 = 0, Mxx = 0, Myy = 0, Mzz = 0, Mxy = 0, Mxz = 0, Myz = 0, Px = 0, Py = 0, Pz = 0;
                    if (c0 >= 0) {
                        R dx, dy, dz, Vx, Vy, Vz;
                        slot_geometry<R>(c0, cxc, cyc, czc, Lx, hLx, Ly, hLy, Lz, hLz, s_px, s_py, s_pz, s_ux, s_uy,
                                         s_uz, s_ox, s_oy, s_oz, sc, dx, dy, dz, Vx, Vy, Vz);
                        const R Bs = (R)B0;
                        Bt = Bs;
                        A0 = Bs * (rho - k15 * (Vx * Vx + Vy * Vy + Vz * Vz));
                        Px = Bs * Vx; Py = Bs * Vy; Pz = Bs * Vz;
                        Mxx = Px * Vx; Myy = Py * Vy; Mzz = Pz * Vz;
                        Mxy = Px * Vy; Mxz = Px * Vz; Myz = Py * Vz;
                    }
                    if (c1 >= 0) {
                        R dx, dy, dz, Vx, Vy, Vz;
                        slot_geometry<R>(c1, cxc, cyc, czc, Lx, hLx, Ly, hLy, Lz, hLz, s_px, s_py, s_pz, s_ux, s_uy,
                                         s_uz, s_ox, s_oy, s_oz, sc, dx, dy, dz, Vx, Vy, Vz);
                        const R Bs = (R)B1;
                        Bt = Bt + Bs;
                        A0 = A0 + Bs * (rho - k15 * (Vx * Vx + Vy * Vy + Vz * Vz));
                        R qx = Bs * Vx, qy = Bs * Vy, qz = Bs * Vz;
                        Px = Px + qx; Py = Py + qy; Pz = Pz + qz;
                        Mxx = Mxx + qx * Vx; Myy = Myy + qy * Vy; Mzz = Mzz + qz * Vz;
                        Mxy = Mxy + qx * Vy; Mxz = Mxz + qx * Vz; Myz = Myz + qy * Vz;
                    }
                    const R omB = (R)1 - Bt;
                    {
                        constexpr R w = (R)W0;
                        R s0 = w * base;
                        R t0 = omega * (s0 - f[0]) - pu0;
                        f[0] = (f[0] + omB * t0) + (w * A0 - Bt * s0);
                        PSM_STORE(0);
                    }
#define PSM_PAIR(Q)                                                                                       \
    pair_psm<R, Q>(f[Q], f[Q + 1], base, Ux, Uy, Uz, (R)(S::SCALED ? bx.fa_scaled[Q / 2] : bx.fa[Q / 2]),     \
                   (R)bx.fs[Q / 2], Q < 7 ? pu1 : pu2, omega, k45, Bt, omB, A0, Mxx, Myy, Mzz, Mxy, Mxz, Myz, Px, \
                   Py, Pz);                                                                                      \
    PSM_STORE(Q);                                                                                                \
    PSM_STORE(Q + 1)
                    PSM_PAIR(1); PSM_PAIR(3); PSM_PAIR(5); PSM_PAIR(7); PSM_PAIR(9);
                    PSM_PAIR(11); PSM_PAIR(13); PSM_PAIR(15); PSM_PAIR(17);
#undef PSM_PAIR
                }
#undef PSM_STORE
            }

            // 5. force and torque of eqs. (21)-(22): sum_q C^solid_{q,s} c_qbar
            // = 2 j - U - U_p(x) per slot (first moment of eq. 19); per-sphere
            // wave sums accumulated per wave in LDS in a fixed order.
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
                    double v[6] = {0, 0, 0, 0, 0, 0};
                    if (Bs != 0.0) {
                        // this cell's share in the collision's precision; the
                        // sums over cells and tiles are FP64
                        R dx, dy, dz, Vx, Vy, Vz;
                        slot_geometry<R>(c, cxc, cyc, czc, Lx, hLx, Ly, hLy, Lz, hLz, s_px, s_py, s_pz, s_ux, s_uy,
                                         s_uz, s_ox, s_oy, s_oz, sc, dx, dy, dz, Vx, Vy, Vz);
                        const R Bh = (R)(S::SCALED ? Bs * (double)kp.h_inv : Bs);
                        const R fx = Bh * (hx - Vx), fy = Bh * (hy - Vy), fz = Bh * (hz - Vz);
                        v[0] = (double)fx;
                        v[1] = (double)fy;
                        v[2] = (double)fz;
                        v[3] = (double)(dy * fz - dz * fy);
                        v[4] = (double)(dz * fx - dx * fz);
                        v[5] = (double)(dx * fy - dy * fx);
                    }
                    int comp;
                    const double sum = wave_sum6(v, lane, comp);
                    if (lane < 6) s_acc[wave][comp][c] += sum;
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
                kp.partial[(long long)(e0 + c) * 6 + k6] = s;
            }
        }
        __syncthreads();
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
        const int nxt = ax.count(), nyt = ay.count(), nzt = az.count();
        const int ntot = nxt * nyt * nzt;
        for (int k = lane; k < ntot; k += 64) {
            int kx = k % nxt, ky = (k / nxt) % nyt, kz = k / (nxt * nyt);
            int t = bx.tile_base + ax.at(kx) + bx.ntx * (ay.at(ky) + bx.nty * az.at(kz));
            int e0 = rp.tile_off[t], e1 = rp.tile_off[t + 1];
            for (int e = e0; e < e1; ++e)
                if (rp.tile_pid[e] == p) {
                    for (int c = 0; c < 6; ++c) acc[c] += rp.partial[(long long)e * 6 + c];
                    break;
                }
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
            if (pos < MAXC && e < bp.cap) bp.tile_pid[e] = p;
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
