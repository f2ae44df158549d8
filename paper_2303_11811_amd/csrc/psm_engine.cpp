// psm_engine.cpp -- host side of the PSM-LBM engine: the C ABI of psm.h.
//
// A context owns no device memory of its own: the caller's workspace is
// carved into per-box ping-pong PDF grids, the global particle table, the
// per-tile candidate lists, the per-(tile, sphere) force partials and a few
// scratch words. Particle uploads go through pinned staging. The time step
// of Sec. 3.1 of the paper (mapping -> PSM kernel -> force reduction) is one
// fused launch over the tiles of all boxes plus one small reduction launch;
// 10-step runs can be replayed from captured HIP graphs. The sphere update of
// Sec. 2.2.2 and the re-binning it needs run on the device as well.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/psm.h"
#include "psm_internal.h"

using namespace psm;

// ---------------------------------------------------------------------------
// Errors

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(PSM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

extern "C" const char* psm_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Launch shapes

static const int kTX[] = {16, 32, 64, 128, 256};
static const int kTZ[] = {1, 2, 4, 8, 16, TZ_MAX};

static bool shape_allowed(int tx, int ty, int tz) {
    bool okx = false, okz = false;
    for (int v : kTX) okx |= (v == tx);
    for (int v : kTZ) okz |= (v == tz);
    return okx && okz && tx * ty == WG;
}

static int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

// Largest number of tiles the bounding box [x-(r+1), x+(r+1)] can touch along
// an axis of L cells cut into tiles of T cells. Its cell range spans at most
// E = floor(2(r+1)) + 2 cells. On a periodic axis whose last
// tile is short (r_last = L - (nt-1)T cells), a range that wraps through it
// touches 1 + ceil((a - r_last)/T) tiles before the wrap and ceil((E - a)/T)
// after it (a cells before the wrap), at most 2 + ceil((E - r_last)/T) in
// all; without a wrap it touches at most 1 + ceil((E-1)/T), which is no more.
static int max_tiles_axis(double rmax, int T, int L) {
    int E = (int)std::floor(2.0 * (rmax + 1.0)) + 2;
    int nt = cdiv(L, T);
    int r_last = L - (nt - 1) * T;
    return std::min(nt, 2 + cdiv(std::max(E - r_last, 0), T));
}

// ---------------------------------------------------------------------------
// Workspace layout

struct Layout {
    size_t off_boxes, off_tbase, off_partbox, off_pt, off_acc, off_fprev, off_prevok, off_tcnt, off_toff, off_tpid, off_tslot,
        off_partial, off_misc, off_statpart, off_scan, total;
    std::vector<size_t> off_grid[2];
    std::vector<int> pblk;
    int T_max;
    long long cap_max;
    int P_total;
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static size_t storage_bytes(int storage) { return storage == PSM_FP64 ? 8 : (storage == PSM_FP32DEV ? 4 : 2); }

static int validate(const psm_box_desc* boxes, int nbox, int storage) {
    if (!boxes || nbox <= 0) return fail(PSM_EINVAL, "need at least one box descriptor");
    if (storage < PSM_FP64 || storage > PSM_FP16DEV) return fail(PSM_EINVAL, "unknown storage %d", storage);
    long long P = 0;
    for (int b = 0; b < nbox; ++b) {
        const psm_box_desc& d = boxes[b];
        if (d.nx < 4 || d.ny < 4 || d.nz < 4) return fail(PSM_EINVAL, "box %d: every dimension must be >= 4", b);
        long long N = (long long)d.nx * d.ny * d.nz;
        if (N > 0x7fffffffLL) return fail(PSM_EINVAL, "box %d: more than 2^31-1 cells", b);
        // byte offsets inside a z-plane are computed in 32-bit signed integers
        // (with the padding to whole 64-cell blocks, FP64 storage bound)
        if ((long long)row_pitch(d.nx) * d.ny * NQ * 8 + 64LL * NQ * 8 >= (1LL << 31))
            return fail(PSM_EINVAL, "box %d: z-planes of 2^31 bytes or more (nx * ny too large)", b);
        if (!(d.tau > 0.5) || !std::isfinite(d.tau)) return fail(PSM_EINVAL, "box %d: tau must be > 1/2", b);
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(d.fext[a])) return fail(PSM_EINVAL, "box %d: non-finite body force", b);
        if (d.max_particles < 0) return fail(PSM_EINVAL, "box %d: max_particles < 0", b);
        if (d.walls_z != 0 && d.walls_z != 1) return fail(PSM_EINVAL, "box %d: walls_z must be 0 or 1", b);
        if ((d.walls_x != 0 && d.walls_x != 1) || (d.walls_y != 0 && d.walls_y != 1))
            return fail(PSM_EINVAL, "box %d: walls_x and walls_y must be 0 or 1", b);
        for (int w = 0; w < 2 && d.walls_z; ++w) {
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(d.wall_u[w][a])) return fail(PSM_EINVAL, "box %d: non-finite wall velocity", b);
            if (d.face_type[w] != PSM_FACE_VELOCITY && d.face_type[w] != PSM_FACE_PRESSURE)
                return fail(PSM_EINVAL, "box %d: unknown face type %d", b, d.face_type[w]);
            if (d.face_type[w] == PSM_FACE_PRESSURE && !(d.face_rho[w] > 0.0 && std::isfinite(d.face_rho[w])))
                return fail(PSM_EINVAL, "box %d: a pressure face needs a positive density", b);
        }
        if (d.mapping != PSM_MAP_LINEAR && d.mapping != PSM_MAP_SUBSAMPLE)
            return fail(PSM_EINVAL, "box %d: unknown mapping %d", b, d.mapping);
        if (d.mapping == PSM_MAP_SUBSAMPLE && (d.subsample_n < 1 || d.subsample_n > 16))
            return fail(PSM_EINVAL, "box %d: subsample_n must be in 1..16", b);
        if (d.max_particles > 0) {
            if (!(d.max_radius >= 1.0) || !std::isfinite(d.max_radius))
                return fail(PSM_EINVAL, "box %d: max_radius must be >= 1", b);
            double need = 2.0 * (d.max_radius + 1.0) + 2.0;
            if (d.nx < need || d.ny < need || d.nz < need)
                return fail(PSM_EINVAL, "box %d: dimensions must be >= 2*(max_radius+1)+2 = %.1f", b, need);
        }
        P += d.max_particles;
    }
    if (P > 0x3fffffffLL) return fail(PSM_EINVAL, "too many particles in total");
    return PSM_OK;
}

static Layout make_layout(const psm_box_desc* boxes, int nbox, int storage) {
    Layout L{};
    size_t s = storage_bytes(storage);
    int P = 0;
    for (int b = 0; b < nbox; ++b) P += boxes[b].max_particles;
    L.P_total = P;
    int Tmax = 0;
    long long capmax = 0;
    for (int tx : kTX)
        for (int tz : kTZ) {
            int ty = WG / tx;
            long long T = 0, cap = 0;
            for (int b = 0; b < nbox; ++b) {
                const psm_box_desc& d = boxes[b];
                T += (long long)cdiv(d.nx, tx) * cdiv(d.ny, ty) * cdiv(d.nz, tz);
                if (d.max_particles > 0)
                    cap += (long long)d.max_particles * max_tiles_axis(d.max_radius, tx, d.nx) *
                           max_tiles_axis(d.max_radius, ty, d.ny) * max_tiles_axis(d.max_radius, tz, d.nz);
            }
            Tmax = (int)std::max<long long>(Tmax, T);
            capmax = std::max(capmax, cap);
        }
    L.T_max = Tmax;
    L.cap_max = std::max<long long>(capmax, 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.off_boxes = take(sizeof(BoxDev) * nbox);
    L.off_tbase = take(sizeof(int) * (nbox + 1));
    L.off_partbox = take(sizeof(int) * std::max(P, 1));
    L.off_pt = take(sizeof(double) * 11 * std::max(P, 1));
    L.off_acc = take(sizeof(double) * 6 * std::max(P, 1) + 64);   // + the device error word
    L.off_fprev = take(sizeof(double) * 6 * std::max(P, 1));
    L.off_prevok = take(sizeof(int) * std::max(P, 1));
    L.off_tcnt = take(sizeof(int) * (size_t)Tmax);
    L.off_toff = take(sizeof(int) * ((size_t)Tmax + 1));
    L.off_tpid = take(sizeof(int) * (size_t)L.cap_max);
    L.off_tslot = take(sizeof(int) * (size_t)L.cap_max);
    L.off_partial = take(sizeof(double) * 6 * (size_t)L.cap_max);
    L.off_misc = take(256);
    L.off_statpart = take(sizeof(double) * 4 * (size_t)stats_blocks() + 64);
    L.off_scan = take(sizeof(int) * 2 * (size_t)scan_chunks(Tmax) + 64);
    for (int p = 0; p < 2; ++p) L.off_grid[p].resize(nbox);
    L.pblk.resize(nbox);
    for (int b = 0; b < nbox; ++b) {
        int pb = cdiv((long long)row_pitch(boxes[b].nx) * boxes[b].ny, BLK);   // 64-cell blocks per z-plane
        L.pblk[b] = pb;
        size_t elems = (size_t)boxes[b].nz * pb * NQ * BLK;
        for (int p = 0; p < 2; ++p) L.off_grid[p][b] = take(s * elems);
    }
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// Context

struct psm_ctx {
    int nbox = 0, storage = 0;
    int map_mode = 0;            // 1 if any box uses sub-division sampling
    float h_scale = 1.0f, h_inv = 1.0f;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L;
    std::vector<psm_box_desc> desc;
    std::vector<BoxDev> box;     // host copy of the device box table
    std::vector<int> np;         // particles set per box
    int P_total = 0;
    TileShape ts{64, 4, 16, 0, 0};
    int T_total = 0;
    int grid = 0;
    int parity = 0;
    bool have_particles_lists = false;
    bool strict_slots = false;      // a third overlap in a cell is an error
    // mass drift check per box: relative tolerance (0 = off) and reference mass (NaN = not taken)
    std::vector<double> drift_tol, ref_mass;
    // device pointers into the workspace
    BoxDev* d_boxes = nullptr;
    int* d_tbase = nullptr;
    int* d_partbox = nullptr;
    Particles P{};
    int *d_tcnt = nullptr, *d_toff = nullptr, *d_tpid = nullptr, *d_tslot = nullptr;
    double* d_partial = nullptr;
    int* d_misc = nullptr;               // [0..1] bin stats, [8..9] dropped (u64),
                                         // [32..39] tile counters of the persistent grid
    int* d_flags = nullptr;              // device error word (FLAG_* bits), right after the force sums
    int* h_flags = nullptr;              // pinned copy of the device error word
    double* d_statpart = nullptr;
    int* d_scan = nullptr;               // scan scratch (chunk sums and maxima)
    // last uploaded positions and radii per box: unchanged geometry keeps the lists
    std::vector<std::vector<double>> last_xr;
    // pinned host staging: two upload halves (reused once their copy has
    // completed, tracked by events) and a read-back area
    double* h_stage = nullptr;
    size_t h_stage_n = 0;
    size_t h_half = 0;               // doubles per upload half
    double* h_read = nullptr;        // read-back area (forces, stats)
    // force read-back at the end of psm_step (psm_set_force_readback): the
    // force sums of all boxes and the error word, copied in one piece
    bool rb_on = false, rb_valid = false;
    double* h_rb = nullptr;          // [6 P_total] sums, then the error word
    hipEvent_t rb_ev = nullptr;
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_next = 0;
    std::vector<std::vector<double>> last_r, last_fr;   // f(r) cache per box
    // graphs of 10 steps, one per starting parity
    bool use_graph = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // graphs of 10 (step + sphere update) pairs, per starting parity, for the
    // time step and scheme they were captured with
    hipGraphExec_t gexec_dyn[2] = {nullptr, nullptr};
    double gdyn_dt[2] = {0.0, 0.0};
    int gdyn_scheme[2] = {-1, -1};
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    long long timed_launches = 0;
    double timed_ms = 0.0;
};

static const int kGraphSteps = 10;

static void drop_graphs(psm_ctx* c) {
    for (int p = 0; p < 2; ++p) {
        if (c->gexec[p]) {
            (void)hipGraphExecDestroy(c->gexec[p]);
            c->gexec[p] = nullptr;
        }
        if (c->gexec_dyn[p]) {
            (void)hipGraphExecDestroy(c->gexec_dyn[p]);
            c->gexec_dyn[p] = nullptr;
        }
    }
}

static int upload_box_table(psm_ctx* c) {
    std::vector<int> tb(c->nbox + 1);
    for (int b = 0; b < c->nbox; ++b) tb[b] = c->box[b].tile_base;
    tb[c->nbox] = c->T_total;
    HIP_TRY(hipMemcpyAsync(c->d_boxes, c->box.data(), sizeof(BoxDev) * c->nbox, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->d_tbase, tb.data(), sizeof(int) * (c->nbox + 1), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));   // the host vectors are pageable temporaries
    return PSM_OK;
}

static void assign_tiles(psm_ctx* c) {
    int base = 0;
    for (int b = 0; b < c->nbox; ++b) {
        BoxDev& bx = c->box[b];
        bx.ntx = cdiv(bx.nx, c->ts.tx);
        bx.nty = cdiv(bx.ny, c->ts.ty);
        bx.ntz = cdiv(bx.nz, c->ts.tz);
        bx.tile_base = base;
        base += bx.ntx * bx.nty * bx.ntz;
    }
    c->T_total = base;
    // force-partial slots: per sphere, one per tile its bounding box can
    // touch at this tile shape (at most the capacity the layout reserves)
    long long pbase = 0;
    for (int b = 0; b < c->nbox; ++b) {
        const psm_box_desc& d = c->desc[b];
        BoxDev& bx = c->box[b];
        bx.pstride = max_tiles_axis(d.max_radius, c->ts.tx, d.nx) * max_tiles_axis(d.max_radius, c->ts.ty, d.ny) *
                     max_tiles_axis(d.max_radius, c->ts.tz, d.nz);
        bx.pbase = (int)pbase;
        pbase += (long long)d.max_particles * bx.pstride;
    }
    int dev = 0, ncu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // one-shot: a workgroup per tile (rounded up to whole XCD rounds);
    // persistent: as many workgroups as fit at once, each walking its tiles
    int full = ((c->T_total + NXCD - 1) / NXCD) * NXCD;
    int g = c->ts.persistent ? std::min(step_blocks_per_cu(c->storage, c->map_mode, c->ts.filter != 0) * ncu, full) : full;
    c->grid = std::max(NXCD, g / NXCD * NXCD);
}

// Rebuild the per-tile candidate lists of all boxes (synchronises).
static int rebuild_lists(psm_ctx* c) {
    // the step kernel must never run on half-built lists
    c->have_particles_lists = false;
    BinParams bp;
    bp.boxes = c->d_boxes;
    bp.part_box = c->d_partbox;
    bp.P = c->P;
    bp.tile_cnt = c->d_tcnt;
    bp.tile_off = c->d_toff;
    bp.tile_pid = c->d_tpid;
    bp.tile_slot = c->d_tslot;
    bp.partial = c->d_partial;
    bp.P_total = c->P_total;
    bp.T_total = c->T_total;
    bp.ts = c->ts;
    bp.cap = c->L.cap_max;
    HIP_TRY(launch_bin(bp, c->d_misc, c->d_scan, c->stream));
    int stats[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(stats, c->d_misc, sizeof stats, hipMemcpyDeviceToHost, c->stream));
    // list flags of earlier builds are void; this build reports its own here
    HIP_TRY(launch_check_lists(c->d_misc, c->L.cap_max, c->d_flags, 0, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (stats[1] > c->L.cap_max)
        return fail(PSM_ECAPACITY, "tile lists need %d entries, capacity %lld", stats[1], c->L.cap_max);
    if (stats[0] > MAXC)
        return fail(PSM_ECAPACITY, "a tile has %d sphere candidates (limit %d): use a smaller tile shape",
                    stats[0], MAXC);
    HIP_TRY(launch_bin_fill(bp, c->stream));
    c->have_particles_lists = true;
    return PSM_OK;
}

// Rebuild the lists without waiting for the device: the counts are checked on
// the device, which replaces the list bits of the error word (the fill and the
// step kernel stay in bounds on capped lists); synchronising calls report them.
static int rebuild_lists_async(psm_ctx* c) {
    BinParams bp;
    bp.boxes = c->d_boxes;
    bp.part_box = c->d_partbox;
    bp.P = c->P;
    bp.tile_cnt = c->d_tcnt;
    bp.tile_off = c->d_toff;
    bp.tile_pid = c->d_tpid;
    bp.tile_slot = c->d_tslot;
    bp.partial = c->d_partial;
    bp.P_total = c->P_total;
    bp.T_total = c->T_total;
    bp.ts = c->ts;
    bp.cap = c->L.cap_max;
    HIP_TRY(launch_bin(bp, c->d_misc, c->d_scan, c->stream));
    HIP_TRY(launch_check_lists(c->d_misc, c->L.cap_max, c->d_flags, 1, c->stream));
    HIP_TRY(launch_bin_fill(bp, c->stream));
    c->have_particles_lists = true;
    return PSM_OK;
}

// Every synchronising call copies the device error word with its read-back
// (sync_with_flags) and reports it afterwards (take_flags), which clears the
// word on the device. A list overflow (device-built lists) or, in strict-slot
// mode, a third overlap makes the context refuse to step until
// psm_set_particles; a bad psm_get_pdfs_at index is an argument error.
static int sync_with_flags(psm_ctx* c) {
    HIP_TRY(hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PSM_OK;
}

static int take_flags(psm_ctx* c) {
    const int f = *c->h_flags;
    if (f == 0) return PSM_OK;
    *c->h_flags = 0;
    HIP_TRY(launch_fill_int(c->d_flags, 1, 0, c->stream));
    if (f & FLAG_LIST_ENTRIES) {
        c->have_particles_lists = false;
        return fail(PSM_ECAPACITY, "the spheres need more tile-list entries than the context holds");
    }
    if (f & FLAG_LIST_TILE) {
        c->have_particles_lists = false;
        return fail(PSM_ECAPACITY, "the spheres put more than %d candidates into a tile: use a smaller tile shape",
                    MAXC);
    }
    if ((f & FLAG_SLOT_OVERFLOW) && c->strict_slots) {
        c->have_particles_lists = false;
        return fail(PSM_ECAPACITY, "strict slots: a cell is overlapped by more than two spheres");
    }
    if (f & FLAG_BAD_CELL)
        return fail(PSM_EINVAL, "psm_get_pdfs_at: a cell index was outside the box (those outputs are NaN)");
    return PSM_OK;
}

extern "C" int psm_workspace_size(const psm_box_desc* boxes, int nbox, int storage, size_t* bytes) {
    if (!bytes) return fail(PSM_EINVAL, "bytes is NULL");
    int rc = validate(boxes, nbox, storage);
    if (rc) return rc;
    Layout L = make_layout(boxes, nbox, storage);
    if (L.cap_max >= (1LL << 31))
        return fail(PSM_EINVAL, "tile lists would need %lld entries (at most 2^31 - 1)", L.cap_max);
    *bytes = L.total;
    return PSM_OK;
}

extern "C" int psm_create(const psm_box_desc* boxes, int nbox, int storage, double fp16_scale, void* hip_stream,
                          void* dev_workspace, size_t workspace_bytes, psm_ctx** out) {
    if (!out) return fail(PSM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(boxes, nbox, storage);
    if (rc) return rc;
    if (!dev_workspace) return fail(PSM_EINVAL, "workspace is NULL");
    if (((uintptr_t)dev_workspace) & 255) return fail(PSM_EINVAL, "workspace must be 256-byte aligned");
    Layout L = make_layout(boxes, nbox, storage);
    if (L.cap_max >= (1LL << 31))
        return fail(PSM_EINVAL, "tile lists would need %lld entries (at most 2^31 - 1)", L.cap_max);
    if (workspace_bytes < L.total)
        return fail(PSM_EINVAL, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);
    if (storage == PSM_FP16DEV) {
        if (fp16_scale == 0.0) fp16_scale = 1024.0;
        int e = 0;
        double m = std::frexp(fp16_scale, &e);
        if (!(fp16_scale > 0.0) || m != 0.5) return fail(PSM_EINVAL, "fp16_scale must be a power of two");
    }

    psm_ctx* c = new psm_ctx();
    c->nbox = nbox;
    c->storage = storage;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)dev_workspace;
    c->L = L;
    c->desc.assign(boxes, boxes + nbox);
    for (int b = 0; b < nbox; ++b)
        if (boxes[b].mapping == PSM_MAP_SUBSAMPLE) c->map_mode = 1;
    if (storage == PSM_FP16DEV) {
        c->h_scale = (float)fp16_scale;
        c->h_inv = (float)(1.0 / fp16_scale);
    }
    c->P_total = L.P_total;
    c->np.assign(nbox, 0);
    c->box.resize(nbox);
    int pb = 0;
    for (int b = 0; b < nbox; ++b) {
        const psm_box_desc& d = boxes[b];
        BoxDev& bx = c->box[b];
        std::memset(&bx, 0, sizeof bx);
        bx.nx = d.nx; bx.ny = d.ny; bx.nz = d.nz;
        bx.N = d.nx * d.ny * d.nz;
        bx.part_base = pb;
        bx.np = 0;
        bx.mapping = d.mapping;
        bx.nsub = d.mapping == PSM_MAP_SUBSAMPLE ? d.subsample_n : 1;
        bx.pitch = row_pitch(d.nx);
        bx.pblk = L.pblk[b];
        bx.plane_elems = (long long)L.pblk[b] * NQ * BLK;
        bx.grid[0] = c->ws + L.off_grid[0][b];
        bx.grid[1] = c->ws + L.off_grid[1][b];
        bx.omega = 1.0 / d.tau;
        bx.pref = 1.0 - 1.0 / (2.0 * d.tau);
        for (int a = 0; a < 3; ++a) bx.g[a] = d.fext[a];
        for (int k = 0; k < 9; ++k) {
            int q = 2 * k + 1;
            double cg = CX[q] * d.fext[0] + CY[q] * d.fext[1] + CZ[q] * d.fext[2];
            bx.fa[k] = 3.0 * bx.pref * wq(q) * cg;
            bx.fa_scaled[k] = bx.fa[k] * (storage == PSM_FP16DEV ? fp16_scale : 1.0);
            bx.fs[k] = 9.0 * bx.pref * wq(q) * cg;
        }
        int dims[3] = {d.nx, d.ny, d.nz};
        for (int a = 0; a < 3; ++a) {
            bx.L[a] = dims[a];
            bx.halfL[a] = 0.5 * dims[a];
        }
        for (int k = 0; k < 16; ++k) bx.sub_off[k] = k < bx.nsub ? (k + 0.5) / bx.nsub - 0.5 : 0.0;
        bx.reach = 0.8660254037844386 * (1.0 - 1.0 / bx.nsub) + 1e-9;
        bx.rho_p = 1.0;
        bx.walls = d.walls_z;
        bx.walls_xy = (d.walls_x ? 1 : 0) | (d.walls_y ? 2 : 0);
        for (int w = 0; w < 2; ++w) {
            bx.face_type[w] = d.walls_z ? d.face_type[w] : FACE_VELOCITY;
            bx.face_rho[w] = bx.face_type[w] == FACE_PRESSURE ? d.face_rho[w] : 1.0;
        }
        for (int w = 0; w < 2; ++w)
            for (int q = 0; q < NQ; ++q) {
                // entering through the bottom face: c_z = +1; through the top: c_z = -1
                bool in = d.walls_z && bx.face_type[w] == FACE_VELOCITY && CZ[q] == (w == 0 ? 1 : -1);
                double cu = CX[q] * d.wall_u[w][0] + CY[q] * d.wall_u[w][1] + CZ[q] * d.wall_u[w][2];
                bx.bw[w][q] = in ? 6.0 * wq(q) * cu : 0.0;
            }
        bx.pw[0] = bx.pref * W0;
        bx.pw[1] = bx.pref * W1;
        bx.pw[2] = bx.pref * W2;
        bx.omega_f = (float)bx.omega;
        for (int a = 0; a < 3; ++a) bx.g_f[a] = (float)bx.g[a];
        for (int k = 0; k < 9; ++k) {
            bx.fa_f[k] = (float)bx.fa[k];
            bx.fs_f[k] = (float)bx.fs[k];
            bx.fa_scaled_f[k] = (float)bx.fa_scaled[k];
        }
        for (int k = 0; k < 3; ++k) bx.pw_f[k] = (float)bx.pw[k];
        {
            // the FP16 form works on scale * d: quadratic terms carry 1/scale
            const double inv_s = storage == PSM_FP16DEV ? 1.0 / fp16_scale : 1.0;
            const double Wc[3] = {W0, W1, W2};
            bx.om1 = 1.0 - bx.omega;
            bx.k15 = 1.5 * inv_s;
            bx.k45 = 4.5 * inv_s;
            for (int c = 0; c < 3; ++c) {
                bx.wk[c] = Wc[c] * bx.k45;
                bx.owk[c] = bx.omega * bx.wk[c];
                bx.ow3[c] = 3.0 * bx.omega * Wc[c];
            }
            bx.om1_f = (float)bx.om1;
            bx.k15_f = (float)bx.k15;
            bx.k45_f = (float)bx.k45;
            for (int c = 0; c < 3; ++c) {
                bx.wk_f[c] = (float)bx.wk[c];
                bx.owk_f[c] = (float)bx.owk[c];
                bx.ow3_f[c] = (float)bx.ow3[c];
            }
        }
        // the FP32 reach test works on centres within a tile extent (at most
        // 256 cells) plus the radius of the tile: a few FP32 ulps of that
        bx.margin32 = 1e-3 + 16.0 * std::ldexp(256.0 + (d.max_particles > 0 ? d.max_radius : 1.0) + 2.0, -24);
        pb += d.max_particles;
    }
    c->d_boxes = (BoxDev*)(c->ws + L.off_boxes);
    c->d_tbase = (int*)(c->ws + L.off_tbase);
    c->d_partbox = (int*)(c->ws + L.off_partbox);
    double* pt = (double*)(c->ws + L.off_pt);
    size_t P1 = std::max(c->P_total, 1);
    double** fields[11] = {&c->P.x, &c->P.y, &c->P.z, &c->P.r, &c->P.fr, &c->P.ux,
                           &c->P.uy, &c->P.uz, &c->P.ox, &c->P.oy, &c->P.oz};
    for (int k = 0; k < 11; ++k) *fields[k] = pt + k * P1;
    c->P.acc = (double*)(c->ws + L.off_acc);
    c->P.fprev = (double*)(c->ws + L.off_fprev);
    c->P.prev_ok = (int*)(c->ws + L.off_prevok);
    c->d_tcnt = (int*)(c->ws + L.off_tcnt);
    c->d_toff = (int*)(c->ws + L.off_toff);
    c->d_tpid = (int*)(c->ws + L.off_tpid);
    c->d_tslot = (int*)(c->ws + L.off_tslot);
    c->d_partial = (double*)(c->ws + L.off_partial);
    c->d_misc = (int*)(c->ws + L.off_misc);
    c->d_flags = (int*)(c->P.acc + 6 * P1);
    c->d_statpart = (double*)(c->ws + L.off_statpart);
    c->d_scan = (int*)(c->ws + L.off_scan);
    c->last_xr.assign(nbox, std::vector<double>());

    int err = PSM_OK;
    auto hip_ok = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && err == PSM_OK) err = fail(PSM_EHIP, "%s: %s", what, hipGetErrorString(e));
    };
    c->h_half = 11 * P1 + 64;
    c->h_stage_n = 2 * c->h_half + 9 * P1 + 64 + 6 * P1 + 64;
    hip_ok(hipHostMalloc((void**)&c->h_stage, sizeof(double) * c->h_stage_n, hipHostMallocDefault), "hipHostMalloc");
    if (err) { delete c; return err; }
    c->h_read = c->h_stage + 2 * c->h_half;
    c->h_flags = (int*)(c->h_read + 9 * P1);   // inside the read area's padding
    *c->h_flags = 0;
    c->h_rb = c->h_read + 9 * P1 + 64;
    {
        const char* e = std::getenv("PSM_STRICT_SLOTS");
        c->strict_slots = e && std::strcmp(e, "1") == 0;
    }
    c->drift_tol.assign(nbox, 0.0);
    c->ref_mass.assign(nbox, std::nan(""));
    for (int h = 0; h < 2; ++h) hip_ok(hipEventCreateWithFlags(&c->stage_ev[h], hipEventDisableTiming), "event");
    hip_ok(hipEventCreateWithFlags(&c->rb_ev, hipEventDisableTiming), "event");
    if (err) { (void)hipHostFree(c->h_stage); delete c; return err; }
    c->last_r.assign(nbox, std::vector<double>());
    c->last_fr.assign(nbox, std::vector<double>());

    std::vector<int> partbox(P1, 0);
    for (int b = 0; b < nbox; ++b)
        for (int p = 0; p < boxes[b].max_particles; ++p) partbox[c->box[b].part_base + p] = b;
    hip_ok(hipMemcpyAsync(c->d_partbox, partbox.data(), sizeof(int) * P1, hipMemcpyHostToDevice, c->stream),
           "upload part_box");
    hip_ok(hipMemsetAsync(c->P.acc, 0, sizeof(double) * 6 * P1 + 64, c->stream), "clear forces and error word");
    hip_ok(hipMemsetAsync(pt, 0, sizeof(double) * 11 * P1, c->stream), "clear particles");
    hip_ok(hipMemsetAsync(c->P.fprev, 0, sizeof(double) * 6 * P1, c->stream), "clear previous forces");
    hip_ok(hipMemsetAsync(c->P.prev_ok, 0, sizeof(int) * P1, c->stream), "clear previous-force flags");
    hip_ok(hipMemsetAsync(c->d_misc, 0, 256, c->stream), "clear counters");
    hip_ok(hipStreamSynchronize(c->stream), "sync");
    if (err) { (void)hipHostFree(c->h_stage); delete c; return err; }

    assign_tiles(c);
    int r2 = upload_box_table(c);
    if (r2 == PSM_OK) r2 = rebuild_lists(c);
    if (r2 != PSM_OK) {
        (void)hipHostFree(c->h_stage);
        delete c;
        return r2;
    }
    *out = c;
    return PSM_OK;
}

extern "C" int psm_destroy(psm_ctx* c) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (int h = 0; h < 2; ++h)
        if (c->stage_ev[h]) (void)hipEventDestroy(c->stage_ev[h]);
    if (c->rb_ev) (void)hipEventDestroy(c->rb_ev);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    delete c;
    return PSM_OK;
}

static int check_box(psm_ctx* c, int box) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (box < 0 || box >= c->nbox) return fail(PSM_EINVAL, "box %d out of range [0,%d)", box, c->nbox);
    return PSM_OK;
}

extern "C" int psm_set_equilibrium(psm_ctx* c, int box, const double* rho, const double* u) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!u) return fail(PSM_EINVAL, "u is NULL");
    HIP_TRY(launch_set_equilibrium(c->storage, c->box[box], c->parity, rho, u, c->h_scale, c->stream));
    c->ref_mass[box] = std::nan("");   // a new state: the drift reference is taken again
    return PSM_OK;
}

extern "C" int psm_set_pdfs(psm_ctx* c, int box, const double* f) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!f) return fail(PSM_EINVAL, "f is NULL");
    HIP_TRY(launch_set_pdfs(c->storage, c->box[box], c->parity, f, c->h_scale, c->stream));
    c->ref_mass[box] = std::nan("");   // a new state: the drift reference is taken again
    return PSM_OK;
}

extern "C" int psm_get_pdfs(psm_ctx* c, int box, double* f) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!f) return fail(PSM_EINVAL, "f is NULL");
    HIP_TRY(launch_get_pdfs(c->storage, c->box[box], c->parity, f, c->h_inv, c->stream));
    return PSM_OK;
}

extern "C" int psm_get_pdfs_at(psm_ctx* c, int box, int ncells, const int* cells, double* out) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (ncells < 0) return fail(PSM_EINVAL, "ncells < 0");
    if (ncells == 0) return PSM_OK;
    if (!cells || !out) return fail(PSM_EINVAL, "cells/out is NULL");
    HIP_TRY(launch_get_pdfs_at(c->storage, c->box[box], c->parity, cells, ncells, out, c->h_inv, c->d_flags,
                               c->stream));
    return PSM_OK;
}

extern "C" int psm_get_macroscopic(psm_ctx* c, int box, double* rho, double* u) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!rho || !u) return fail(PSM_EINVAL, "rho/u is NULL");
    HIP_TRY(launch_macroscopic(c->storage, c->box[box], c->parity, rho, u, c->h_inv, c->stream));
    return PSM_OK;
}

// f(r) = V_a - r + 1/2 of eq. (26), with V_a the closed form of eq. (27):
// the integral of sqrt(r^2 - x^2 - y^2) over the unit square.
static double solid_fraction_offset(double r) {
    double r2 = r * r;
    double s = std::sqrt(r2 - 0.5);
    double Va = (1.0 / 12.0 - r2) * std::atan((0.5 * s) / (0.5 - r2)) + s / 3.0 +
                (r2 - 1.0 / 12.0) * std::atan(0.5 / s) - (4.0 / 3.0) * r * r2 * std::atan(0.25 / (r * s));
    return Va - r + 0.5;
}

static double wrap_coord(double v, double L) {
    double w = v - L * std::floor(v / L);
    if (w >= L) w -= L;   // v slightly below a multiple of L
    if (w < 0.0) w = 0.0;
    return w;
}

extern "C" int psm_set_particles(psm_ctx* c, int box, int n, const double* x, const double* r, const double* U,
                                 const double* omega) {
    int rc = check_box(c, box);
    if (rc) return rc;
    const psm_box_desc& d = c->desc[box];
    if (n < 0) return fail(PSM_EINVAL, "n < 0");
    if (n > d.max_particles) return fail(PSM_ECAPACITY, "box %d holds at most %d particles (got %d)", box, d.max_particles, n);
    if (n > 0 && (!x || !r || !U)) return fail(PSM_EINVAL, "x/r/U is NULL");
    for (int p = 0; p < n; ++p) {
        if (!(r[p] >= 1.0 && r[p] <= d.max_radius))
            return fail(PSM_EINVAL, "particle %d: radius %g outside [1, %g]", p, r[p], d.max_radius);
        const int walled[3] = {d.walls_x, d.walls_y, d.walls_z};
        const int dims3[3] = {d.nx, d.ny, d.nz};
        for (int a = 0; a < 3; ++a)
            if (walled[a] && !(x[3 * p + a] >= r[p] + 1.0 && x[3 * p + a] <= dims3[a] - r[p] - 1.0))
                return fail(PSM_EINVAL, "particle %d: centre closer than r + 1 to a wall", p);
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(x[3 * p + a]) || !std::isfinite(U[3 * p + a]) ||
                (omega && !std::isfinite(omega[3 * p + a])))
                return fail(PSM_EINVAL, "particle %d: non-finite input", p);
        }
    }
    // staging: 11 SoA columns of length n (stride m), in the order of the
    // device table, in the upload half whose previous copy has completed
    int m = d.max_particles;
    int h = c->stage_next;
    c->stage_next ^= 1;
    HIP_TRY(hipEventSynchronize(c->stage_ev[h]));
    double* st = c->h_stage + (size_t)h * c->h_half;
    double Lx = d.nx, Ly = d.ny, Lz = d.nz;
    std::vector<double>& lr = c->last_r[box];
    std::vector<double>& lf = c->last_fr[box];
    lr.resize(n, -1.0);
    lf.resize(n, 0.0);
    for (int p = 0; p < n; ++p) {
        st[0 * m + p] = wrap_coord(x[3 * p + 0], Lx);
        st[1 * m + p] = wrap_coord(x[3 * p + 1], Ly);
        st[2 * m + p] = wrap_coord(x[3 * p + 2], Lz);
        st[3 * m + p] = r[p];
        if (lr[p] != r[p]) {   // f(r) only depends on r
            lr[p] = r[p];
            lf[p] = solid_fraction_offset(r[p]);
        }
        st[4 * m + p] = lf[p];
        for (int a = 0; a < 3; ++a) {
            st[(5 + a) * m + p] = U[3 * p + a];
            st[(8 + a) * m + p] = omega ? omega[3 * p + a] : 0.0;
        }
    }
    // the 11 device columns are P_total apart: one strided copy moves them all
    int pb = c->box[box].part_base;
    size_t P1 = (size_t)std::max(c->P_total, 1);
    if (n > 0)
        HIP_TRY(hipMemcpy2DAsync(c->P.x + pb, sizeof(double) * P1, st, sizeof(double) * m, sizeof(double) * n, 11,
                                 hipMemcpyHostToDevice, c->stream));
    // new velocities: velocity Verlet starts again from this state
    HIP_TRY(launch_fill_int(c->P.prev_ok + pb, m, 0, c->stream));
    bool np_changed = c->np[box] != n;
    if (np_changed) {
        int* npst = (int*)(st + 11 * (size_t)m);
        *npst = n;
        HIP_TRY(hipMemcpyAsync(&c->d_boxes[box].np, npst, sizeof(int), hipMemcpyHostToDevice, c->stream));
    }
    HIP_TRY(hipEventRecord(c->stage_ev[h], c->stream));
    // positions (wrapped) and radii decide the tile lists; velocities do not
    bool same_geometry = c->have_particles_lists && !np_changed && (size_t)4 * n == c->last_xr[box].size();
    for (int k = 0; k < 4 && same_geometry; ++k)
        same_geometry = std::memcmp(c->last_xr[box].data() + (size_t)k * n, st + (size_t)k * m,
                                    sizeof(double) * n) == 0;
    c->box[box].np = n;
    c->np[box] = n;
    if (same_geometry) return PSM_OK;
    std::vector<double>& xr = c->last_xr[box];
    xr.resize((size_t)4 * n);
    for (int k = 0; k < 4; ++k) std::memcpy(xr.data() + (size_t)k * n, st + (size_t)k * m, sizeof(double) * n);
    // lists rebuilt on the device without waiting: an overflow is reported by
    // the next synchronising call
    rc = rebuild_lists_async(c);
    if (rc != PSM_OK) xr.clear();
    return rc;
}

// Upload some columns of the sphere table of box `box` (n spheres, the
// current count) through the pinned staging: cols[k] (host, row-major (n,3))
// goes to the three device columns first_col[k] .. first_col[k] + 2. Checks
// each value while it stages it (finite; a position column also keeps r + 1
// from the walls and is wrapped into the box) and enqueues nothing when one
// fails. Asynchronous.
static int upload_columns(psm_ctx* c, int box, int n, const double* const* cols, const int* first_col, int ncols) {
    const psm_box_desc& d = c->desc[box];
    const int m = d.max_particles;
    const int h = c->stage_next;
    c->stage_next ^= 1;
    HIP_TRY(hipEventSynchronize(c->stage_ev[h]));
    double* st = c->h_stage + (size_t)h * c->h_half;
    const double L[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
    const int walled[3] = {d.walls_x, d.walls_y, d.walls_z};
    const std::vector<double>& r = c->last_r[box];
    const int pb = c->box[box].part_base;
    const size_t P1 = (size_t)std::max(c->P_total, 1);
    double* dev_cols[11] = {c->P.x, c->P.y, c->P.z, c->P.r, c->P.fr, c->P.ux, c->P.uy, c->P.uz, c->P.ox, c->P.oy, c->P.oz};
    for (int k = 0; k < ncols; ++k) {
        double* sk = st + (size_t)3 * k * m;
        const double* v = cols[k];
        if (first_col[k] == 0) {
            for (int p = 0; p < n; ++p)
                for (int a = 0; a < 3; ++a) {
                    const double xa = v[3 * p + a];
                    if (!std::isfinite(xa)) return fail(PSM_EINVAL, "particle %d: non-finite position", p);
                    if (walled[a] && !(xa >= r[p] + 1.0 && xa <= L[a] - r[p] - 1.0))
                        return fail(PSM_EINVAL, "particle %d: centre closer than r + 1 to a wall", p);
                    sk[(size_t)a * m + p] = wrap_coord(xa, L[a]);
                }
        } else if (v) {
            for (int p = 0; p < n; ++p)
                for (int a = 0; a < 3; ++a) {
                    const double va = v[3 * p + a];
                    if (!std::isfinite(va)) return fail(PSM_EINVAL, "particle %d: non-finite velocity", p);
                    sk[(size_t)a * m + p] = va;
                }
        } else {
            for (int a = 0; a < 3; ++a) std::fill(sk + (size_t)a * m, sk + (size_t)a * m + n, 0.0);
        }
    }
    // the three device columns of each are P_total apart: one strided copy
    for (int k = 0; k < ncols && n > 0; ++k)
        HIP_TRY(hipMemcpy2DAsync(dev_cols[first_col[k]] + pb, sizeof(double) * P1, st + (size_t)3 * k * m,
                                 sizeof(double) * m, sizeof(double) * n, 3, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(c->stage_ev[h], c->stream));
    return PSM_OK;
}

static int check_update_args(psm_ctx* c, int box, int n) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (n != c->np[box])
        return fail(PSM_EINVAL, "box %d holds %d spheres (psm_set_particles), got %d", box, c->np[box], n);
    return PSM_OK;
}

extern "C" int psm_set_particle_positions(psm_ctx* c, int box, int n, const double* x) {
    int rc = check_update_args(c, box, n);
    if (rc) return rc;
    if (n > 0 && !x) return fail(PSM_EINVAL, "x is NULL");
    const double* cols[1] = {x};
    const int first[1] = {0};
    if ((rc = upload_columns(c, box, n, cols, first, 1))) return rc;
    c->last_xr[box].clear();   // positions changed outside psm_set_particles
    return rebuild_lists_async(c);
}

extern "C" int psm_set_particle_velocities(psm_ctx* c, int box, int n, const double* U, const double* omega) {
    int rc = check_update_args(c, box, n);
    if (rc) return rc;
    if (n > 0 && !U) return fail(PSM_EINVAL, "U is NULL");
    const double* cols[2] = {U, omega};
    const int first[2] = {5, 8};
    if ((rc = upload_columns(c, box, n, cols, first, 2))) return rc;
    // new velocities: velocity Verlet starts again from this state
    HIP_TRY(launch_fill_int(c->P.prev_ok + c->box[box].part_base, c->desc[box].max_particles, 0, c->stream));
    return PSM_OK;
}

static int step_params(psm_ctx* c, int parity, StepParams& kp) {
    kp.boxes = c->d_boxes;
    kp.box_tile_base = c->d_tbase;
    kp.nbox = c->nbox;
    kp.P = c->P;
    kp.tile_off = c->d_toff;
    kp.tile_pid = c->d_tpid;
    kp.tile_slot = c->d_tslot;
    kp.partial = c->d_partial;
    kp.T_total = c->T_total;
    kp.tx = c->ts.tx; kp.ty = c->ts.ty; kp.tz = c->ts.tz;
    kp.parity = parity;
    kp.h_scale = c->h_scale;
    kp.h_inv = c->h_inv;
    kp.flags = c->d_flags;
    kp.queue = c->ts.persistent ? c->d_misc + 32 : nullptr;   // ints 32..39 of the counter block
    return PSM_OK;
}

static ReduceParams reduce_params(psm_ctx* c) {
    ReduceParams rp;
    rp.boxes = c->d_boxes;
    rp.nbox = c->nbox;
    rp.part_box = c->d_partbox;
    rp.P = c->P;
    rp.tile_off = c->d_toff;
    rp.tile_pid = c->d_tpid;
    rp.partial = c->d_partial;
    rp.P_total = c->P_total;
    rp.ts = c->ts;
    return rp;
}

// Kernel timing keeps a fixed pool of events (created when timing is turned
// on, so that none is created inside a timed loop). When the pool is full,
// the recorded pairs are folded into the totals: the last recorded event is
// waited for (every earlier one is then complete) and the pool starts over.
constexpr size_t kEvPool = 256;

static int create_events(psm_ctx* c) {
    if (c->ev.size() >= kEvPool) return PSM_OK;
    while (c->ev.size() < kEvPool) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->ev.push_back(e);
    }
    // record each event once here: a first record costs more than later ones,
    // and the first timed steps should not pay for it
    for (hipEvent_t e : c->ev) HIP_TRY(hipEventRecord(e, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PSM_OK;
}

static int fold_events(psm_ctx* c) {
    if (c->ev_used >= 2) HIP_TRY(hipEventSynchronize(c->ev[c->ev_used - 1]));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->timed_ms += ms;
        c->timed_launches++;
    }
    c->ev_used = 0;
    return PSM_OK;
}

static hipEvent_t next_event(psm_ctx* c) {
    if (c->ev_used == kEvPool && fold_events(c) != PSM_OK) return nullptr;
    if (c->ev_used == c->ev.size() && create_events(c) != PSM_OK) return nullptr;
    return c->ev[c->ev_used++];
}

static int enqueue_step(psm_ctx* c, bool timed) {
    StepParams kp;
    step_params(c, c->parity, kp);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = next_event(c);
        e1 = e0 ? next_event(c) : nullptr;
        if (!e0 || !e1) return fail(PSM_EHIP, "timing events: %s", g_err.c_str());
        HIP_TRY(hipEventRecord(e0, c->stream));
    }
    // the persistent grid's tile counters start at zero (a kernel, not a
    // memset: the step may be captured into a graph)
    if (kp.queue) HIP_TRY(launch_fill_int(kp.queue, NXCD, 0, c->stream));
    HIP_TRY(launch_step(c->storage, c->map_mode, c->ts.filter != 0, kp, c->grid, c->stream));
    if (timed) HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(launch_reduce(reduce_params(c), c->stream));
    c->parity ^= 1;
    c->rb_valid = false;
    return PSM_OK;
}

static int build_graph(psm_ctx* c, int start_parity) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int saved = c->parity;
    c->parity = start_parity;
    int rc = PSM_OK;
    for (int s = 0; s < kGraphSteps && rc == PSM_OK; ++s) rc = enqueue_step(c, false);
    c->parity = saved;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != PSM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(PSM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec[start_parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PSM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return PSM_OK;
}

extern "C" int psm_step(psm_ctx* c, int nsteps) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(PSM_EINVAL, "nsteps < 0");
    if (!c->have_particles_lists) return fail(PSM_ESTATE, "tile lists are not built");
    // graph replays enqueue steps without passing through enqueue_step
    if (nsteps > 0) c->rb_valid = false;
    int left = nsteps;
    if (c->use_graph && !c->timing) {
        while (left >= kGraphSteps) {
            int p = c->parity;
            if (!c->gexec[p]) {
                int rc = build_graph(c, p);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(c->gexec[p], c->stream));
            left -= kGraphSteps;   // an even count: the parity is unchanged
        }
    }
    for (; left > 0; --left) {
        int rc = enqueue_step(c, c->timing);
        if (rc) return rc;
    }
    if (c->rb_on && nsteps > 0) {
        // the force sums of every box and the error word, one contiguous copy
        const size_t P1 = (size_t)std::max(c->P_total, 1);
        HIP_TRY(hipMemcpyAsync(c->h_rb, c->P.acc, sizeof(double) * 6 * P1 + sizeof(int), hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipEventRecord(c->rb_ev, c->stream));
        c->rb_valid = true;
    }
    return PSM_OK;
}

extern "C" int psm_set_force_readback(psm_ctx* c, int enable) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    c->rb_on = enable != 0;
    c->rb_valid = false;
    return PSM_OK;
}

extern "C" int psm_get_forces(psm_ctx* c, int box, double* F, double* T) {
    int rc = check_box(c, box);
    if (rc) return rc;
    int n = c->np[box];
    if (n == 0) return (rc = sync_with_flags(c)) ? rc : take_flags(c);
    if (!F || !T) return fail(PSM_EINVAL, "F/T is NULL");
    const double* st;
    if (c->rb_valid) {
        // the copy psm_step made: wait for it, not for work enqueued after it
        HIP_TRY(hipEventSynchronize(c->rb_ev));
        int f = *(const int*)(c->h_rb + 6 * (size_t)std::max(c->P_total, 1));
        if (!c->strict_slots) f &= ~FLAG_SLOT_OVERFLOW;
        // an error bit: report it the usual way, from the end of the stream
        if (f && ((rc = sync_with_flags(c)) || (rc = take_flags(c)))) return rc;
        st = c->h_rb + 6LL * c->box[box].part_base;
    } else {
        HIP_TRY(hipMemcpyAsync(c->h_read, c->P.acc + 6LL * c->box[box].part_base, sizeof(double) * 6 * n,
                               hipMemcpyDeviceToHost, c->stream));
        if ((rc = sync_with_flags(c)) || (rc = take_flags(c))) return rc;
        st = c->h_read;
    }
    for (int p = 0; p < n; ++p)
        for (int a = 0; a < 3; ++a) {
            F[3 * p + a] = st[6 * p + a];
            T[3 * p + a] = st[6 * p + 3 + a];
        }
    return PSM_OK;
}

extern "C" int psm_get_solid_fraction(psm_ctx* c, int box, double* B, int* pid) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!B || !pid) return fail(PSM_EINVAL, "B/pid is NULL");
    unsigned long long* dropped = (unsigned long long*)(c->d_misc + 8);
    HIP_TRY(hipMemsetAsync(dropped, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(launch_map_dense(c->box[box], c->P, c->d_toff, c->d_tpid, c->ts, B, pid, dropped, c->stream));
    return PSM_OK;
}

extern "C" int psm_get_stats(psm_ctx* c, int box, double* mass, double* momentum, long long* slot_overflows) {
    int rc = check_box(c, box);
    if (rc) return rc;
    double* out = c->d_statpart + 4 * stats_blocks();
    HIP_TRY(launch_stats(c->storage, c->box[box], c->parity, c->h_inv, c->d_statpart, out, c->stream));
    unsigned long long* dropped = (unsigned long long*)(c->d_misc + 8);
    HIP_TRY(hipMemsetAsync(dropped, 0, sizeof(unsigned long long), c->stream));
    HIP_TRY(launch_map_dense(c->box[box], c->P, c->d_toff, c->d_tpid, c->ts, nullptr, nullptr, dropped, c->stream));
    double* st = c->h_read;
    HIP_TRY(hipMemcpyAsync(st, out, sizeof(double) * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(st + 4, dropped, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync_with_flags(c)) || (rc = take_flags(c))) return rc;
    if (mass) *mass = st[0];
    if (momentum)
        for (int a = 0; a < 3; ++a) momentum[a] = st[1 + a];
    unsigned long long dr;
    std::memcpy(&dr, st + 4, sizeof dr);
    if (slot_overflows) *slot_overflows = (long long)dr;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(st[k])) return fail(PSM_ENONFINITE, "box %d: non-finite mass or momentum", box);
    if (c->drift_tol[box] > 0.0) {
        // the first totals after the check is enabled or the state is set are the reference
        if (std::isnan(c->ref_mass[box])) {
            c->ref_mass[box] = st[0];
        } else {
            const double ref = c->ref_mass[box], rel = std::fabs(st[0] - ref) / std::fabs(ref);
            if (!(rel <= c->drift_tol[box]))
                return fail(PSM_EDRIFT, "box %d: mass %.17g drifted from %.17g by %.3g (relative), above %.3g", box,
                            st[0], ref, rel, c->drift_tol[box]);
        }
    }
    return PSM_OK;
}

extern "C" int psm_set_drift_check(psm_ctx* c, int box, double rel_tol) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return fail(PSM_EINVAL, "rel_tol must be >= 0 and finite");
    const psm_box_desc& d = c->desc[box];
    if (rel_tol > 0.0 && d.walls_z)
        for (int w = 0; w < 2; ++w)
            if (d.face_type[w] == PSM_FACE_PRESSURE || d.wall_u[w][2] != 0.0)
                return fail(PSM_EINVAL, "box %d: a pressure face or a face with a normal velocity exchanges mass; "
                                        "the drift check needs a closed or periodic box", box);
    c->drift_tol[box] = rel_tol;
    c->ref_mass[box] = std::nan("");
    return PSM_OK;
}

extern "C" int psm_set_strict_slots(psm_ctx* c, int enable) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    // overlaps seen before the switch do not count
    HIP_TRY(hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (*c->h_flags & FLAG_SLOT_OVERFLOW) {
        *c->h_flags &= ~FLAG_SLOT_OVERFLOW;
        HIP_TRY(launch_fill_int(c->d_flags, 1, *c->h_flags, c->stream));
    }
    *c->h_flags = 0;
    c->strict_slots = enable != 0;
    return PSM_OK;
}

extern "C" int psm_set_dynamics(psm_ctx* c, int box, double density_ratio, const double* accel) {
    int rc = check_box(c, box);
    if (rc) return rc;
    if (!(density_ratio > 0.0) || !std::isfinite(density_ratio))
        return fail(PSM_EINVAL, "density ratio must be positive and finite");
    double a[3] = {0.0, 0.0, 0.0};
    if (accel)
        for (int k = 0; k < 3; ++k) {
            if (!std::isfinite(accel[k])) return fail(PSM_EINVAL, "non-finite acceleration");
            a[k] = accel[k];
        }
    BoxDev& bx = c->box[box];
    bx.rho_p = density_ratio;
    for (int k = 0; k < 3; ++k) bx.accel[k] = a[k];
    return upload_box_table(c);
}

// Sphere update and device-side re-binning (no host state is touched, so
// that it can be captured).
static int enqueue_integrate(psm_ctx* c, double dt, int scheme) {
    IntParams ip;
    ip.boxes = c->d_boxes;
    ip.part_box = c->d_partbox;
    ip.P = c->P;
    ip.P_total = c->P_total;
    ip.dt = dt;
    HIP_TRY(launch_integrate(scheme == PSM_EULER ? SCHEME_EULER : SCHEME_VERLET, ip, c->stream));
    return rebuild_lists_async(c);
}

static int check_dynamics_args(psm_ctx* c, double dt, int scheme) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PSM_EINVAL, "dt must be positive and finite");
    if (scheme != PSM_EULER && scheme != PSM_VERLET) return fail(PSM_EINVAL, "unknown scheme %d", scheme);
    if (!c->have_particles_lists) return fail(PSM_ESTATE, "no valid particle set");
    return PSM_OK;
}

extern "C" int psm_integrate(psm_ctx* c, double dt, int scheme) {
    int rc = check_dynamics_args(c, dt, scheme);
    if (rc) return rc;
    rc = enqueue_integrate(c, dt, scheme);
    // the host copies of positions are stale from here on
    for (auto& v : c->last_xr) v.clear();
    return rc;
}

static int build_dyn_graph(psm_ctx* c, int start_parity, double dt, int scheme) {
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int saved = c->parity;
    c->parity = start_parity;
    int rc = PSM_OK;
    for (int s = 0; s < kGraphSteps && rc == PSM_OK; ++s) {
        rc = enqueue_step(c, false);
        if (rc == PSM_OK) rc = enqueue_integrate(c, dt, scheme);
    }
    c->parity = saved;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != PSM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(PSM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (c->gexec_dyn[start_parity]) (void)hipGraphExecDestroy(c->gexec_dyn[start_parity]);
    c->gexec_dyn[start_parity] = nullptr;
    e = hipGraphInstantiate(&c->gexec_dyn[start_parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PSM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    c->gdyn_dt[start_parity] = dt;
    c->gdyn_scheme[start_parity] = scheme;
    return PSM_OK;
}

extern "C" int psm_run(psm_ctx* c, int nsteps, double dt, int scheme) {
    int rc = check_dynamics_args(c, dt, scheme);
    if (rc) return rc;
    if (nsteps < 0) return fail(PSM_EINVAL, "nsteps < 0");
    // graph replays enqueue steps without passing through enqueue_step
    if (nsteps > 0) c->rb_valid = false;
    int left = nsteps;
    if (c->use_graph && !c->timing) {
        while (left >= kGraphSteps) {
            int p = c->parity;
            if (!c->gexec_dyn[p] || c->gdyn_dt[p] != dt || c->gdyn_scheme[p] != scheme) {
                rc = build_dyn_graph(c, p, dt, scheme);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(c->gexec_dyn[p], c->stream));
            left -= kGraphSteps;   // an even count: the parity is unchanged
        }
    }
    for (; left > 0; --left) {
        rc = enqueue_step(c, c->timing);
        if (rc == PSM_OK) rc = enqueue_integrate(c, dt, scheme);
        if (rc) return rc;
    }
    if (nsteps > 0)
        for (auto& v : c->last_xr) v.clear();
    return PSM_OK;
}

extern "C" int psm_get_particles(psm_ctx* c, int box, double* x, double* U, double* omega) {
    int rc = check_box(c, box);
    if (rc) return rc;
    int n = c->np[box];
    if (n == 0 || (!x && !U && !omega)) return (rc = sync_with_flags(c)) ? rc : take_flags(c);
    size_t P1 = (size_t)std::max(c->P_total, 1);
    int pb = c->box[box].part_base;
    // columns x y z (0-2), ux uy uz (5-7), ox oy oz (8-10) of the device table
    double* st = c->h_read;
    HIP_TRY(hipMemcpy2DAsync(st, sizeof(double) * n, c->P.x + pb, sizeof(double) * P1, sizeof(double) * n, 3,
                             hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpy2DAsync(st + 3 * (size_t)n, sizeof(double) * n, c->P.ux + pb, sizeof(double) * P1,
                             sizeof(double) * n, 6, hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync_with_flags(c)) || (rc = take_flags(c))) return rc;
    double* outs[3] = {x, U, omega};
    for (int k = 0; k < 3; ++k) {
        if (!outs[k]) continue;
        for (int p = 0; p < n; ++p)
            for (int a = 0; a < 3; ++a) outs[k][3 * p + a] = st[(size_t)(3 * k + a) * n + p];
    }
    return PSM_OK;
}

extern "C" int psm_set_launch(psm_ctx* c, int tx, int ty, int tz, int flags) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (!shape_allowed(tx, ty, tz)) return fail(PSM_EINVAL, "launch shape %dx%dx%d not allowed", tx, ty, tz);
    if (flags & ~(PSM_LAUNCH_PERSISTENT | PSM_LAUNCH_FILTER)) return fail(PSM_EINVAL, "unknown launch flags %d", flags);
    HIP_TRY(hipStreamSynchronize(c->stream));
    TileShape old = c->ts;
    c->ts = TileShape{tx, ty, tz, (flags & PSM_LAUNCH_PERSISTENT) ? 1 : 0, (flags & PSM_LAUNCH_FILTER) ? 1 : 0};
    assign_tiles(c);
    int rc = upload_box_table(c);
    if (rc == PSM_OK) rc = rebuild_lists(c);
    if (rc != PSM_OK) {
        std::string msg = g_err;
        c->ts = old;
        assign_tiles(c);
        if (upload_box_table(c) == PSM_OK) (void)rebuild_lists(c);
        g_err = msg;
        return rc;
    }
    drop_graphs(c);
    return PSM_OK;
}

static int launch_flags(const TileShape& t) {
    return (t.persistent ? PSM_LAUNCH_PERSISTENT : 0) | (t.filter ? PSM_LAUNCH_FILTER : 0);
}

extern "C" int psm_get_launch(psm_ctx* c, int* tx, int* ty, int* tz, int* flags) {
    if (!c || !tx || !ty || !tz) return fail(PSM_EINVAL, "NULL argument");
    *tx = c->ts.tx; *ty = c->ts.ty; *tz = c->ts.tz;
    if (flags) *flags = launch_flags(c->ts);
    return PSM_OK;
}

extern "C" int psm_set_graph(psm_ctx* c, int enable) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    c->use_graph = enable != 0;
    if (!c->use_graph) drop_graphs(c);
    return PSM_OK;
}

extern "C" int psm_set_timing(psm_ctx* c, int enable) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (enable) {
        int rc = create_events(c);
        if (rc) return rc;
    }
    c->timing = enable != 0;
    return PSM_OK;
}

extern "C" int psm_get_timing(psm_ctx* c, long long* launches, double* total_ms) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    int rc = fold_events(c);
    if (rc) return rc;
    if (launches) *launches = c->timed_launches;
    if (total_ms) *total_ms = c->timed_ms;
    return PSM_OK;
}

extern "C" int psm_pattern_copy(psm_ctx* c, int shifted, int nrep, double* ms) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (shifted != 0 && shifted != 1) return fail(PSM_EINVAL, "shifted must be 0 or 1");
    if (nrep < 1) return fail(PSM_EINVAL, "nrep < 1");
    if (!ms) return fail(PSM_EINVAL, "ms is NULL");
    StepParams kp;
    step_params(c, c->parity, kp);
    hipEvent_t e[2] = {nullptr, nullptr};
    HIP_TRY(hipEventCreate(&e[0]));
    hipError_t err = hipEventCreate(&e[1]);
    if (err == hipSuccess) err = hipEventRecord(e[0], c->stream);
    for (int i = 0; i < nrep && err == hipSuccess; ++i)
        err = launch_pattern_copy(c->storage, shifted != 0, kp, c->grid, c->stream);
    if (err == hipSuccess) err = hipEventRecord(e[1], c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e[1]);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e[0], e[1]);
    (void)hipEventDestroy(e[0]);
    if (e[1]) (void)hipEventDestroy(e[1]);
    if (err != hipSuccess) return fail(PSM_EHIP, "psm_pattern_copy: %s", hipGetErrorString(err));
    *ms = (double)t / nrep;
    return PSM_OK;
}

extern "C" int psm_reset_timing(psm_ctx* c) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->ev_used = 0;
    c->timed_launches = 0;
    c->timed_ms = 0.0;
    return PSM_OK;
}

// ---------------------------------------------------------------------------
// Autotune cache: the launch picked for a class of contexts, kept for the
// process and, if PSM_TUNE_CACHE names a file, across processes (one line per
// entry: key, tx, ty, tz, flags, ms per step).

struct TuneEntry {
    TileShape ts;
    double ms;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;
static bool g_tune_loaded = false;

// The class of a context: GPU architecture, storage form, mapping, and per
// box its dimensions, walls and sphere volume fraction (rounded to a power
// of two in hundredths): the quantities the best launch depends on.
static std::string tune_key(psm_ctx* c) {
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s|s%d|m%d|n%d", arch.c_str(), c->storage, c->map_mode, c->nbox);
    std::string k = buf;
    for (int b = 0; b < c->nbox; ++b) {
        const psm_box_desc& d = c->desc[b];
        double vol = 0.0;
        for (double r : c->last_r[b]) vol += 4.18879020478639098 * r * r * r;
        const double frac = vol / ((double)d.nx * d.ny * d.nz);
        const int cls = frac <= 0.0 ? -1 : (int)std::lround(std::log2(std::max(frac * 100.0, 1e-3)));
        std::snprintf(buf, sizeof buf, "|%dx%dx%d:%d%d%d:%d", d.nx, d.ny, d.nz, d.walls_x, d.walls_y, d.walls_z, cls);
        k += buf;
    }
    return k;
}

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("PSM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[4096];
    TuneEntry e{};
    while (std::fscanf(f, "%4095s %d %d %d %d %d %lf", key, &e.ts.tx, &e.ts.ty, &e.ts.tz, &e.ts.persistent,
                       &e.ts.filter, &e.ms) == 7)
        if (shape_allowed(e.ts.tx, e.ts.ty, e.ts.tz)) g_tune[key] = e;
    std::fclose(f);
}

static void tune_store_locked(const std::string& key, const TuneEntry& e) {
    g_tune[key] = e;
    const char* path = std::getenv("PSM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %d %.6f\n", key.c_str(), e.ts.tx, e.ts.ty, e.ts.tz, e.ts.persistent, e.ts.filter,
                 e.ms);
    std::fclose(f);
}

extern "C" int psm_clear_tune_cache(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = true;   // entries of the file are not read again in this process
    return PSM_OK;
}

static int autotune_timed(psm_ctx* c, int trial_steps, TileShape& best, double& best_t);

extern "C" int psm_autotune(psm_ctx* c, int trial_steps, int* tx, int* ty, int* tz, int* flags,
                            double* best_ms) {
    if (!c) return fail(PSM_EINVAL, "ctx is NULL");
    if (trial_steps < 1) return fail(PSM_EINVAL, "trial_steps must be >= 1");
    const std::string key = tune_key(c);
    TuneEntry hit{};
    bool cached = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            hit = it->second;
            cached = true;
        }
    }
    TileShape best;
    double best_t = 0.0;
    int rc;
    if (cached) {
        best = hit.ts;
        best_t = hit.ms;
        rc = psm_set_launch(c, best.tx, best.ty, best.tz, launch_flags(best));
        if (rc) return rc;
    } else {
        rc = autotune_timed(c, trial_steps, best, best_t);
        if (rc) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_store_locked(key, TuneEntry{best, best_t});
    }
    if (tx) *tx = best.tx;
    if (ty) *ty = best.ty;
    if (tz) *tz = best.tz;
    if (flags) *flags = launch_flags(best);
    if (best_ms) *best_ms = best_t;
    return PSM_OK;
}

// Time every allowed launch on the context and keep the fastest (see psm.h).
static int autotune_timed(psm_ctx* c, int trial_steps, TileShape& best_out, double& best_ms_out) {
    bool was_timing = c->timing, was_graph = c->use_graph;
    c->timing = false;
    c->use_graph = false;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PSM_EHIP, "hipEventCreate failed");
    }
    // ms per step of the current launch shape: two untimed steps, then nsteps timed
    auto time_current = [&](int nsteps, double& per) -> int {
        int rc = psm_step(c, 2);
        if (rc) return rc;
        if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(PSM_EHIP, "hipEventRecord failed");
        if ((rc = psm_step(c, nsteps))) return rc;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return fail(PSM_EHIP, "timing event failed");
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(PSM_EHIP, "hipEventElapsedTime failed");
        per = ms / nsteps;
        return PSM_OK;
    };
    auto time_shape = [&](const TileShape& ts, int nsteps, double& per) -> int {
        int rc = psm_set_launch(c, ts.tx, ts.ty, ts.tz, launch_flags(ts));
        return rc ? rc : time_current(nsteps, per);
    };
    struct Cand {
        TileShape ts;
        double t;
    };
    std::vector<Cand> cands;
    int maxdim = 0;
    for (auto& d : c->desc) maxdim = std::max(maxdim, d.nx);
    int rc = PSM_OK;
    // first round: every shape once
    for (int fl = 0; fl < 4 && !rc; ++fl)
        for (int txv : kTX) {
            // tiles much wider than the widest box only idle lanes
            if (txv > 2 * std::max(maxdim, 16)) continue;
            for (int tzv : kTZ) {
                TileShape ts{txv, WG / txv, tzv, (fl & PSM_LAUNCH_PERSISTENT) != 0, (fl & PSM_LAUNCH_FILTER) != 0};
                if (psm_set_launch(c, ts.tx, ts.ty, ts.tz, fl) != PSM_OK) continue;   // not allowed here
                double per = 0.0;
                if ((rc = time_current(trial_steps, per))) break;
                cands.push_back({ts, per});
            }
        }
    // second round: the fastest few again, interleaved, with twice the steps,
    // so that one noisy trial does not decide
    TileShape best = c->ts;
    double best_t = 1e300;
    if (!rc && !cands.empty()) {
        std::stable_sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.t < b.t; });
        const int K = std::min<int>(4, (int)cands.size());
        std::vector<double> tot(K, 0.0);
        for (int rep = 0; rep < 2 && !rc; ++rep)
            for (int i = 0; i < K && !rc; ++i) {
                double per = 0.0;
                rc = time_shape(cands[i].ts, 2 * trial_steps, per);
                tot[i] += per;
            }
        for (int i = 0; i < K && !rc; ++i)
            if (tot[i] / 2 < best_t) {
                best_t = tot[i] / 2;
                best = cands[i].ts;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = was_timing;
    c->use_graph = was_graph;
    if (rc) return rc;
    if (cands.empty()) return fail(PSM_EINVAL, "no launch shape is allowed for these boxes");
    rc = psm_set_launch(c, best.tx, best.ty, best.tz, launch_flags(best));
    if (rc) return rc;
    best_out = best;
    best_ms_out = best_t;
    return PSM_OK;
}

extern "C" int psm_field_stats_noalloc(const double* f, long long ncells, double* out, void* hip_stream) {
    if (ncells < 0) return fail(PSM_EINVAL, "ncells < 0");
    if (ncells > noalloc_max_cells())
        return fail(PSM_EINVAL, "psm_field_stats_noalloc: %lld cells, at most %lld (fixed scratch)", ncells,
                    noalloc_max_cells());
    if ((ncells > 0 && !f) || !out) return fail(PSM_EINVAL, "f/out is NULL");
    HIP_TRY(launch_field_stats_noalloc(f, ncells, out, (hipStream_t)hip_stream));
    return PSM_OK;
}

extern "C" int psm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
    if (!src || !dst) return fail(PSM_EINVAL, "NULL pointer");
    if (bytes % 16) return fail(PSM_EINVAL, "bytes must be a multiple of 16");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(PSM_EINVAL, "pointers must be 16-byte aligned");
    const char* s = (const char*)src;
    char* d = (char*)dst;
    if (s < d + bytes && d < s + bytes) return fail(PSM_EINVAL, "buffers overlap");
    HIP_TRY(launch_stream_copy(src, dst, bytes, (hipStream_t)hip_stream));
    return PSM_OK;
}
