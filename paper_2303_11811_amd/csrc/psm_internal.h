// psm_internal.h -- structures and device helpers shared by the engine's
// kernels and host code (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psm {

constexpr int NQ = 19;
constexpr int WG = 256;          // threads per workgroup of the step kernel
constexpr int NWAVE = WG / 64;   // 64-wide wavefronts per workgroup
constexpr int MAXC = 64;         // sphere candidates per tile staged in LDS
constexpr int TZ_MAX = 32;   // largest cells per thread along z of a tile
constexpr int NXCD = 8;          // MI355X: 8 accelerator complex dies, 32 CUs each
#ifndef PSM_BLK
#define PSM_BLK 64
#endif
constexpr int BLK = PSM_BLK;     // cells per PDF storage block (one wavefront)

// D3Q19 velocity set in the canonical order of the ABI (psm.h). Directions
// come in inverse pairs (2k-1, 2k) for k = 1..9.
constexpr int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
__host__ __device__ constexpr double wq(int q) { return q == 0 ? W0 : (q <= 6 ? W1 : W2); }

// Per-box constants, stored in device memory and read with scalar loads.
struct BoxDev {
    int nx, ny, nz, N;
    int ntx, nty, ntz, tile_base;   // tiles per axis, first global tile
    int part_base, np, mapping, nsub;
    // force partials of a sphere: slots pbase + (local id) * pstride + k for
    // the k-th tile of its bounding box (pstride bounds the tiles a sphere of
    // this box can touch at the current tile shape)
    int pstride, pbase;
    // PDF storage: each z-plane holds pblk blocks of 64 cells (pitch*ny
    // rounded up); a block stores its 19 directions one after another, 64
    // values each. Cell (x, y) of a plane is in-plane cell x + pitch*y.
    int pitch;                      // row pitch in cells, see row_pitch()
    int pblk;                       // blocks per z-plane
    long long plane_elems;          // values per z-plane, pblk * 19 * 64
    void* grid[2];                  // ping-pong PDF grids, nz * plane_elems values
    double omega, pref;             // 1/tau, 1 - 1/(2 tau)
    double g[3];                    // body-force density
    // Forcing constants of eq. (8) with the Guo prefactor, precomputed on the
    // host so that the kernel reads them from scalar registers:
    //   F_q = fa[k] + fs[k] (c_q.U) - pw[class] 3 (U.g) for the pair k = (q, q+1),
    //   F_qbar = -fa[k] + fs[k] (c_q.U) - pw[class] 3 (U.g).
    double fa[9], fs[9];            // 3 pref w (c.g), 9 pref w (c.g)
    double fa_scaled[9];            // fa times the FP16 storage scale
    double pw[3];                   // pref w for the rest, axis and diagonal weights
    // Collision constants per weight class c (rest, axis, diagonal) with the
    // FP16 storage scale s folded in (s = 1 otherwise):
    //   k15 = 1.5/s, k45 = 4.5/s, wk[c] = W_c k45, owk[c] = omega W_c k45, ow3[c] = 3 omega W_c
    double om1, k15, k45, wk[3], owk[3], ow3[3];
    // FP32 copies of the collision constants for the deviation forms
    float omega_f, g_f[3], fa_f[9], fs_f[9], fa_scaled_f[9], pw_f[3];
    float om1_f, k15_f, k45_f, wk_f[3], owk_f[3], ow3_f[3];
    // rounding margin (cells) of the step kernel's FP32 reach test
    double margin32;
    // Geometry constants for the minimum image and the sub-sample test.
    double L[3], halfL[3];          // box lengths and their halves
    double sub_off[16];             // (k + 1/2)/nsub - 1/2, k < nsub
    double reach;                   // sqrt(3) (1/2 - 1/(2 nsub)) + 1e-9
    // Sphere dynamics of the box: density ratio to the fluid and external
    // acceleration (gravity minus buoyancy) used by the integrator.
    double rho_p;
    double accel[3];
    // Faces at z = 0 and z = nz instead of periodicity (walls != 0). On a
    // velocity face w a population q entering a boundary cell is the one the
    // cell sent against the face (direction inv_dir(q)) plus bw[w][q] =
    // 6 w_q (c_q . u_w) (half-way bounce-back); on a pressure face it is
    // minus that population plus 2 w_q (face_rho[w] + 4.5 (c_q.u)^2 - 1.5 u.u)
    // with u the cell's post-collision velocity (anti-bounce-back).
    int walls;
    int walls_xy;                   // bit 0: resting walls at x = 0, nx; bit 1: at y = 0, ny
    int face_type[2];               // FACE_VELOCITY or FACE_PRESSURE
    double face_rho[2];
    double bw[2][NQ];
};
enum { FACE_VELOCITY = 0, FACE_PRESSURE = 1 };

// Opposite direction: the pairs (1,2), (3,4), ..., (17,18) are opposite.
__host__ __device__ constexpr int inv_dir(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

// Global particle table, SoA, indexed by global particle id.
struct Particles {
    double *x, *y, *z, *r, *fr, *ux, *uy, *uz, *ox, *oy, *oz;
    double* acc;     // [P][6]: F (3), T (3) of the last step
    double* fprev;   // [P][6]: total force and torque of the previous integration (velocity Verlet)
    int* prev_ok;    // [P]: 1 once fprev holds a value
};

struct TileShape {
    int tx, ty, tz;
    int persistent;   // 1: occupancy-sized grid walking the tiles; 0: one workgroup per tile
    int filter;       // 1: per-wave candidate filter before the per-cell mapping
};

// ---------------------------------------------------------------------------
// Tiles of one axis touched by a particle's bounding box.
// The box along the axis covers cells [lo, hi] (unwrapped, hi - lo + 1 <= L).
// Wrapped into [0, L) it is one or two cell segments; their tiles form at most
// two contiguous tile ranges [a0,a1] and [b0,b1] (b empty if b1 < b0), with no
// tile listed twice. Every caller walks them in the same order.
struct AxisTiles {
    int a0, a1, b0, b1;
    __host__ __device__ int count() const { return (a1 - a0 + 1) + (b1 >= b0 ? b1 - b0 + 1 : 0); }
    __host__ __device__ int at(int k) const {
        int na = a1 - a0 + 1;
        return k < na ? a0 + k : b0 + (k - na);
    }
};

__host__ __device__ inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__host__ __device__ inline AxisTiles axis_tiles(int lo, int hi, int L, int T, int nt) {
    AxisTiles r;
    if (lo >= 0 && hi < L) {
        r.a0 = lo / T; r.a1 = hi / T; r.b0 = 0; r.b1 = -1;
        return r;
    }
    int s0, s1, u0, u1;   // segment [s0, L-1] and [0, u1]
    if (lo < 0) { s0 = lo + L; u1 = hi; }
    else { s0 = lo; u1 = hi - L; }
    (void)u0; (void)s1;
    int ta0 = s0 / T, tb1 = u1 / T;
    if (tb1 >= ta0) { r.a0 = 0; r.a1 = nt - 1; r.b0 = 0; r.b1 = -1; }
    else { r.a0 = ta0; r.a1 = nt - 1; r.b0 = 0; r.b1 = tb1; }
    return r;
}

// Cell range of the bounding box [x - (r+1), x + (r+1)] along one axis.
__host__ __device__ inline void aabb_cells(double x, double r, int& lo, int& hi) {
    lo = (int)floor(x - (r + 1.0));
    hi = (int)floor(x + (r + 1.0));
}

// Row pitch of the PDF layout: a row that does not fill whole 64-cell
// blocks is padded to the next block boundary when that costs at most 1/8 of
// the row, so that every row of a tile starts on a block and a wave's loads
// and stores of one direction stay in one block (or two, for a shift in x).
// Narrower rows are packed back to back.
__host__ __device__ inline int row_pitch(int nx) {
    int up = (nx + BLK - 1) / BLK * BLK;
    return 8LL * up <= 9LL * nx ? up : nx;
}

// Element index of direction q of cell (x, y, z) in a box's PDF grid.
__host__ __device__ inline long long pdf_index(const BoxDev& b, int q, int x, int y, int z) {
    int s = x + b.pitch * y;
    return (long long)z * b.plane_elems + (long long)(s / BLK) * (NQ * BLK) + q * BLK + (s % BLK);
}

// ---------------------------------------------------------------------------
// Minimum image of one displacement component into [-L/2, L/2)
// (hL = L/2, exact).
__host__ __device__ inline double min_image(double d, double L, double hL) {
    // two selects (no branch): the conditions exclude each other
    double r = d >= hL ? d - L : d;
    return d < -hL ? d + L : r;
}

// Overlap fraction of a sphere (radius r, f(r) = fr) with the cell whose
// centre lies at displacement (dx, dy, dz) from the sphere centre.
// Linear approximation (Sec. 2.3.2, eq. 26): eps = f(r) - (|d| - r), overlap
// iff eps > 0, capped at 1. No fused multiply-add, so that the fraction is
// reproducible bit for bit.
__device__ inline double overlap_linear(double dx, double dy, double dz, double r, double fr) {
#pragma clang fp contract(off)
    double d2 = dx * dx + dy * dy + dz * dz;
    double lim = r + fr + 1e-9;
    if (d2 > lim * lim) return 0.0;
    double eps = fr - (sqrt(d2) - r);
    if (eps <= 0.0) return 0.0;
    return eps < 1.0 ? eps : 1.0;
}

// Sub-division sampling: fraction of the nsub^3 points at offsets off[k] =
// (k+1/2)/nsub - 1/2 that lie inside the sphere (|s| <= r). Cells farther
// than r + reach from the centre hold no sample inside, cells nearer than
// r - reach hold only inside samples. The test is discontinuous: no fused
// multiply-add, evaluation order ((sx sx + sy sy) + sz sz).
template <class OffPtr>
__device__ inline double overlap_subsample(double dx, double dy, double dz, double r, int nsub, OffPtr off,
                                           double reach) {
#pragma clang fp contract(off)
    double d2 = dx * dx + dy * dy + dz * dz;
    double hi = r + reach;
    if (d2 > hi * hi) return 0.0;
    double lo = r - reach;
    if (lo > 0.0 && d2 < lo * lo) return 1.0;
    double r2 = r * r;
    int inside = 0;
    for (int kz = 0; kz < nsub; ++kz) {
        double sz = dz + off[kz];
        for (int ky = 0; ky < nsub; ++ky) {
            double sy = dy + off[ky];
            for (int kx = 0; kx < nsub; ++kx) {
                double sx = dx + off[kx];
                double s2 = sx * sx + sy * sy + sz * sz;
                inside += (s2 <= r2) ? 1 : 0;
            }
        }
    }
    return (double)inside / ((double)nsub * nsub * nsub);
}

// Two-slot list of one cell (Sec. 3.1.1 stores at most two fractions per
// cell). A candidate is stronger with a larger fraction, ties broken by the
// smaller particle id; a third overlap drops the weakest and is counted.
struct Slots {
    int c0, c1;      // candidate index (or particle id), -1 if empty
    int p0, p1;      // particle id used for ordering
    double B0, B1;
    int dropped;
};

__device__ inline bool stronger(double Ba, int pa, double Bb, int pb) {
    return Ba > Bb || (Ba == Bb && pa < pb);
}

__device__ inline void slots_init(Slots& s) {
    s.c0 = s.c1 = -1; s.p0 = s.p1 = 0x7fffffff; s.B0 = s.B1 = 0.0; s.dropped = 0;
}

__device__ inline void slots_insert(Slots& s, int c, int p, double B) {
    if (s.c0 < 0) { s.c0 = c; s.p0 = p; s.B0 = B; return; }
    if (s.c1 < 0) { s.c1 = c; s.p1 = p; s.B1 = B; return; }
    s.dropped++;
    // the weaker of the two kept slots
    bool w1 = stronger(s.B0, s.p0, s.B1, s.p1);
    if (w1) {
        if (stronger(B, p, s.B1, s.p1)) { s.c1 = c; s.p1 = p; s.B1 = B; }
    } else {
        if (stronger(B, p, s.B0, s.p0)) { s.c0 = c; s.p0 = p; s.B0 = B; }
    }
}

// Ascending particle id, then the B > 1 renormalisation of Sec. 2.3.
__device__ inline void slots_finish(Slots& s) {
    if (s.c1 >= 0 && s.p0 > s.p1) {
        int tc = s.c0; s.c0 = s.c1; s.c1 = tc;
        int tp = s.p0; s.p0 = s.p1; s.p1 = tp;
        double tb = s.B0; s.B0 = s.B1; s.B1 = tb;
    }
    if (s.c1 >= 0) {
        double sum = s.B0 + s.B1;
        if (sum > 1.0) { s.B0 = s.B0 / sum; s.B1 = s.B1 / sum; }
    }
}

// ---------------------------------------------------------------------------
// Launch parameters (passed by value) and launchers of psm_kernels.hip.

struct StepParams {
    const BoxDev* boxes;
    const int* box_tile_base;   // [nbox+1]
    int nbox;
    Particles P;
    const int* tile_off;        // [T+1]
    const int* tile_pid;        // [entries] global particle ids
    const int* tile_slot;       // [entries] force-partial slot of each entry
    double* partial;            // [slots][6]
    int T_total;
    int tx, ty, tz;
    int parity;
    float h_scale, h_inv;       // FP16 storage scale and its inverse (1 otherwise)
    int* flags;                 // device error word: |= FLAG_SLOT_OVERFLOW when a cell meets a third sphere
    int* queue;                 // [NXCD] tile counters of the persistent grid (zeroed before the launch), or null
};

struct ReduceParams {
    const BoxDev* boxes;
    int nbox;
    const int* part_box;        // [P] box of each global particle slot
    Particles P;
    const int* tile_off;
    const int* tile_pid;
    const double* partial;
    int P_total;
    TileShape ts;
};

struct BinParams {
    const BoxDev* boxes;
    const int* part_box;
    Particles P;
    int* tile_cnt;
    int* tile_off;
    int* tile_pid;
    int* tile_slot;             // [entries] force-partial slot of each entry
    double* partial;            // [slots][6], zeroed for an entry a full list drops
    int P_total;
    int T_total;
    TileShape ts;
    long long cap;              // entries tile_pid holds
};

// Sphere integration (explicit Euler or velocity Verlet) of every particle.
enum { SCHEME_EULER = 0, SCHEME_VERLET = 1 };
struct IntParams {
    const BoxDev* boxes;
    const int* part_box;
    Particles P;
    int P_total;
    double dt;
};

hipError_t launch_step(int storage, int map, bool filt, const StepParams& kp, int grid, hipStream_t st);
hipError_t launch_pattern_copy(int storage, bool shifted, const StepParams& kp, int grid, hipStream_t st);
int step_blocks_per_cu(int storage, int map, bool filt);
hipError_t launch_reduce(const ReduceParams& rp, hipStream_t st);
int scan_chunks(int n);
hipError_t launch_bin(const BinParams& bp, int* stats, int* scratch, hipStream_t st);
hipError_t launch_bin_fill(const BinParams& bp, hipStream_t st);
hipError_t launch_set_pdfs(int storage, const BoxDev& bx, int parity, const double* f, float scale, hipStream_t st);
hipError_t launch_set_equilibrium(int storage, const BoxDev& bx, int parity, const double* rho, const double* u,
                                  float scale, hipStream_t st);
hipError_t launch_get_pdfs(int storage, const BoxDev& bx, int parity, double* f, float inv, hipStream_t st);
hipError_t launch_get_pdfs_at(int storage, const BoxDev& bx, int parity, const int* cells, int ncells, double* out,
                              float inv, int* flags, hipStream_t st);
hipError_t launch_macroscopic(int storage, const BoxDev& bx, int parity, double* rho, double* u, float inv,
                              hipStream_t st);
hipError_t launch_map_dense(const BoxDev& bx, const Particles& P, const int* tile_off, const int* tile_pid,
                            TileShape ts, double* B, int* pid, unsigned long long* dropped, hipStream_t st);
int stats_blocks();
hipError_t launch_stats(int storage, const BoxDev& bx, int parity, float inv, double* part, double* out,
                        hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
hipError_t launch_integrate(int scheme, const IntParams& ip, hipStream_t st);
// Bits of the device error word of a context, set by kernels and read and
// cleared by the host at its next synchronising call.
enum {
    FLAG_LIST_ENTRIES = 1,    // the tile lists need more entries than the context holds
    FLAG_LIST_TILE = 2,       // a tile lists more than MAXC spheres
    FLAG_SLOT_OVERFLOW = 4,   // a step met a cell overlapped by more than two spheres
    FLAG_BAD_CELL = 8         // psm_get_pdfs_at was given a cell index outside the box
};
// Replace the list bits of err: FLAG_LIST_ENTRIES if the lists need more than
// cap entries, FLAG_LIST_TILE if a tile lists more than MAXC spheres (report =
// 0: clear the list bits only)
hipError_t launch_check_lists(const int* stats, long long cap, int* err, int report, hipStream_t st);
hipError_t launch_fill_int(int* a, long long n, int v, hipStream_t st);
// FP64 mass and momentum of a canonical field [19][N] into out[4] (device),
// with the partial sums in the library's static per-GPU array
long long noalloc_max_cells();
hipError_t launch_field_stats_noalloc(const double* f, long long N, double* out, hipStream_t st);

}  // namespace psm
