/*
 * psm.h -- C ABI of the MI355X (gfx950) engine for the hot path of the
 * partially-saturated-cells lattice Boltzmann method (PSM-LBM) of
 * Kemmler et al., "Efficiency and scalability of fully-resolved
 * fluid-particle simulations on heterogeneous CPU-GPU architectures"
 * (arXiv 2303.11811).
 *
 * One time step (Sec. 3.1 of the paper, the GPU part of its time loop):
 *   sphere -> cell solid-fraction mapping (Sec. 2.3.2, eqs. 25-27),
 *   D3Q19 SRT stream-collide with PSM coupling (Sec. 2.1 eqs. 1-8,
 *   Sec. 2.3 eqs. 17-20), and the per-particle hydrodynamic force and
 *   torque reduction (Sec. 2.3 eqs. 21-22).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every call returns 0 (PSM_OK) or a negative PSM_E* code and never
 *   throws. psm_last_error() returns a thread-local text of the last failure.
 * - Argument checks happen on the host before anything is enqueued; a bad
 *   argument returns PSM_EINVAL and leaves the context unchanged. What only
 *   the device can see (a cell index given in device memory, tile lists built
 *   on the device, a third sphere overlapping a cell) sets a device error
 *   word that the next synchronising call of the context (psm_get_forces,
 *   psm_get_stats, psm_get_particles) reports and clears; the kernels stay in
 *   bounds meanwhile. (With the force read-back on, psm_get_forces reports the
 *   word as the step's copy saw it; see psm_set_force_readback.)
 * - Lattice units: dx = dt = 1, rho_0 = 1, c_s^2 = 1/3. Boxes are periodic
 *   along every axis without walls (psm_box_desc.walls_x, walls_y, walls_z).
 * - Cells: index n = x + nx*(y + ny*z); cell (i,j,k) has its centre at
 *   (i+1/2, j+1/2, k+1/2) in [0,nx) x [0,ny) x [0,nz).
 * - PDFs: canonical layout [19][N] (q-major), FP64, pre-collision state
 *   f(x,t) of eq. (1). Direction order q: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z;
 *   7..18 = (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0),(+1,0,+1),(-1,0,-1),
 *   (+1,0,-1),(-1,0,+1),(0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).
 *   Weights 1/3, 1/18 (axes), 1/36 (diagonals).
 * - Ownership: the caller owns all device memory (one workspace allocation,
 *   e.g. a torch tensor) and the HIP stream. The library owns only its kernels,
 *   HIP graphs and a pinned host staging buffer, all released by psm_destroy.
 * - Pointer kinds: "device" arguments are HIP device pointers and the work is
 *   enqueued on the context's stream (asynchronous); "host" arguments are
 *   ordinary host pointers. Calls marked "synchronises" wait for the stream.
 * - Concurrency: calls on one context are not thread-safe. Use one context
 *   per stream.
 */
#ifndef PSM_H
#define PSM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum psm_status {
    PSM_OK = 0,
    PSM_EINVAL = -1,      /* invalid argument (checked on the host) */
    PSM_EHIP = -2,        /* a HIP runtime call failed; text kept in psm_last_error */
    PSM_ECAPACITY = -3,   /* more particles / tile candidates than the context holds */
    PSM_ENONFINITE = -4,  /* non-finite mass or momentum found by psm_get_stats */
    PSM_EDRIFT = -5,      /* mass drifted beyond the tolerance of psm_set_drift_check */
    PSM_ESTATE = -6       /* call not valid in the current state */
};

/* PDF storage. FP64 stores f and computes in FP64. The deviation forms store
 * d = f - w_q (FP16 as scale*d with a power-of-two scale) and compute the
 * collision and each cell's force and torque share in FP32; the force and
 * torque sums over cells and the mass and momentum sums stay FP64. */
enum psm_storage { PSM_FP64 = 0, PSM_FP32DEV = 1, PSM_FP16DEV = 2 };

/* Boundary type of a z face (psm_box_desc.face_type). */
enum psm_face { PSM_FACE_VELOCITY = 0, PSM_FACE_PRESSURE = 1 };

/* Solid-fraction mapping (Sec. 2.3.2): the linear approximation of eq. (26),
 * or sub-division sampling with subsample_n^3 points per cell. */
enum psm_mapping { PSM_MAP_LINEAR = 0, PSM_MAP_SUBSAMPLE = 1 };

typedef struct psm_box_desc {
    int nx, ny, nz;         /* cells per axis, each >= 4 and >= 2*(max_radius+1)+2 */
    double tau;             /* relaxation time, > 1/2 (eq. 3); nu = (tau-1/2)/3 (eq. 4) */
    double fext[3];         /* body-force density f^ext (eqs. 7-8) */
    int max_particles;      /* capacity of this box's particle table (>= 0) */
    double max_radius;      /* largest sphere radius that will be set (>= 1) */
    int mapping;            /* psm_mapping */
    int subsample_n;        /* samples per axis for PSM_MAP_SUBSAMPLE (1..16) */
    int walls_z;            /* 0: periodic in z; 1: bounded by the faces z = 0 and z = nz (cell
                               faces), each of the type face_type (bottom first) */
    double wall_u[2][3];    /* velocity faces: face velocity u_w; half-way bounce-back with the
                               moving-wall term 6 w_q (c_q . u_w): no-slip for u_w = 0, a moving
                               wall for a tangential u_w, a velocity inflow/outflow for a normal one */
    int face_type[2];       /* psm_face (walls_z = 1) */
    double face_rho[2];     /* pressure faces: density rho_w > 0; anti-bounce-back
                               f_qbar = -f~_q + 2 w_q (rho_w + 4.5 (c_q.u)^2 - 1.5 u.u), u the boundary
                               cell's post-collision velocity */
    int walls_x, walls_y;   /* 1: resting no-slip walls at x = 0 and x = nx (y = 0, y = ny) instead of
                               periodicity (half-way bounce-back); they take precedence over a z face
                               for a population crossing both */
} psm_box_desc;

typedef struct psm_ctx psm_ctx;

/* Bytes of device workspace a context over these boxes needs (host-only call).
 * boxes: host array of nbox descriptors. bytes: host output. */
int psm_workspace_size(const psm_box_desc* boxes, int nbox, int storage, size_t* bytes);

/* Create a context. The workspace (device, >= psm_workspace_size bytes,
 * 256-byte aligned) is carved into PDF grids, particle tables, tile lists and
 * force partials; it must outlive the context and is not freed by it.
 * fp16_scale: power of two used by PSM_FP16DEV (ignored otherwise; 0 selects
 * 1024). hip_stream: hipStream_t (may be NULL for the default stream). The
 * PDF state is undefined until psm_set_equilibrium or psm_set_pdfs. */
int psm_create(const psm_box_desc* boxes, int nbox, int storage, double fp16_scale,
               void* hip_stream, void* dev_workspace, size_t workspace_bytes, psm_ctx** out);

/* Destroy the context (waits for its stream). Does not free the workspace. */
int psm_destroy(psm_ctx* ctx);

/* Initialise box `box` to the equilibrium of eq. (5): f_q = E_q(rho, u).
 * rho: device [N] FP64 or NULL for rho = 1; u: device [3][N] FP64. */
int psm_set_equilibrium(psm_ctx* ctx, int box, const double* rho, const double* u);

/* Set the pre-collision PDFs f(x,t) of box `box`. f: device [19][N] FP64.
 * Deviation storage rounds d = f - w_q to FP32 / FP16 (round to nearest even). */
int psm_set_pdfs(psm_ctx* ctx, int box, const double* f);

/* Read the pre-collision PDFs f(x,t) of box `box` into f: device [19][N] FP64. */
int psm_get_pdfs(psm_ctx* ctx, int box, double* f);

/* Read f(x,t) at ncells cells. cells: device [ncells] int cell indices, each
 * in [0,N); out: device [19][ncells] FP64. The indices are only visible to the
 * device: an index outside [0,N) reads nothing, its 19 outputs are NaN, and
 * the next synchronising call returns PSM_EINVAL. */
int psm_get_pdfs_at(psm_ctx* ctx, int box, int ncells, const int* cells, double* out);

/* Density and velocity of eqs. (6)-(7) (U includes the f^ext/2 shift).
 * rho: device [N] FP64; u: device [3][N] FP64. */
int psm_get_macroscopic(psm_ctx* ctx, int box, double* rho, double* u);

/* Set the spheres of box `box` (Sec. 3.1.1: positions, radii, then linear and
 * angular velocities). Host arrays, row-major: x (n,3), r (n), U (n,3),
 * omega (n,3) (NULL omega = 0); they are copied before the call returns.
 * Positions are wrapped into the box. Radii must lie in [1, max_radius]; along
 * an axis with walls every centre needs r + 1 <= x_a <= n_a - r - 1. The
 * library computes f(r) of eq. (26) in FP64 and uploads through pinned staging.
 * When positions or radii differ from the previous call it rebuilds the
 * per-tile candidate lists on the device. Nothing waits for the device: if
 * a tile would list more candidates than the kernel stages, its list is cut
 * (the steps stay in bounds, their results are not valid) and the next
 * synchronising call returns PSM_ECAPACITY, after which the context refuses
 * to step until a valid set is given. PSM_ECAPACITY at once if
 * n > max_particles. */
int psm_set_particles(psm_ctx* ctx, int box, int n, const double* x, const double* r,
                      const double* U, const double* omega);

/* Update only the positions (host (n,3)) of the spheres of box `box`, with n
 * the count of the last psm_set_particles; radii, velocities and the velocity
 * Verlet state are kept. Positions are wrapped and checked as there; the tile
 * lists are rebuilt on the device. Asynchronous (a host that integrates the
 * spheres can upload the next positions while the current step runs: the
 * upload is ordered after the step on the stream). Overflows are reported as
 * for psm_set_particles. */
int psm_set_particle_positions(psm_ctx* ctx, int box, int n, const double* x);

/* Update only the velocities U and omega (host (n,3); NULL omega = 0) of the
 * spheres of box `box`, n as above; no re-binning. Velocity Verlet starts
 * again from these velocities. Asynchronous. */
int psm_set_particle_velocities(psm_ctx* ctx, int box, int n, const double* U, const double* omega);

/* Advance every box by nsteps time steps: per step, fused mapping +
 * stream-collide + force/torque partial sums (one launch over the tiles of all
 * boxes) and the per-particle reduction. With graphs enabled, runs of 10 steps
 * replay a captured HIP graph. Asynchronous. */
int psm_step(psm_ctx* ctx, int nsteps);

/* Hydrodynamic force and torque of eqs. (21)-(22) on every sphere of box
 * `box` from the last executed step. F, T: host (n,3) FP64 (n = particles set).
 * Synchronises and reports the device error word (see the conventions). Before
 * any step: zeros. With the force read-back on (psm_set_force_readback) and
 * no step enqueued since the last psm_step, it waits only for the copy that
 * psm_step made, not for work enqueued after it. */
int psm_get_forces(psm_ctx* ctx, int box, double* F, double* T);

/* Force read-back for a host that integrates the spheres (the per-step
 * force transfer to the host of Sec. 3.2). enable != 0: every psm_step ends
 * by copying the force and torque sums of all boxes and the device error word
 * into pinned host memory (one copy, 48 B per sphere the context can hold,
 * i.e. max_particles summed over the boxes); psm_get_forces
 * then waits for that copy only, so that a position upload and its re-binning
 * enqueued after the step run while the host reads the forces and updates
 * the velocities. The error word is the one the copy saw: an overflow raised
 * by such a re-binning is reported by the psm_get_forces after the next step
 * (that step runs on the cut lists and stays in bounds). An error bit in the
 * copy makes psm_get_forces synchronise as without the read-back. Off by
 * default; enable = 0 turns it off. PSM_EINVAL for a NULL ctx. */
int psm_set_force_readback(psm_ctx* ctx, int enable);

/* Solid fractions of the current particles (the mapping of the step, in FP64;
 * the FP16-deviation step evaluates the linear approximation in FP32, within
 * about 1e-6 of these): B: device [2][N] FP64, pid: device [2][N] int
 * (box-local particle id, -1 for an empty slot). Slots hold the two largest
 * fractions in ascending id, renormalised to sum 1 where they exceed 1
 * (Sec. 2.3). */
int psm_get_solid_fraction(psm_ctx* ctx, int box, double* B, int* pid);

/* FP64 totals of the current state of box `box`: mass sum_x sum_q f,
 * momentum sum_x sum_q f c_q (host double[3], may be NULL), and the number of
 * dropped third-or-later overlaps of the current mapping (may be NULL).
 * Synchronises and reports the device error word. PSM_ENONFINITE if mass or
 * momentum is not finite; PSM_EDRIFT (outputs still written) if the drift
 * check of the box is on and the mass moved away from its reference. */
int psm_get_stats(psm_ctx* ctx, int box, double* mass, double* momentum, long long* slot_overflows);

/* Mass drift watchdog of box `box`. The method conserves mass (eq. 2 moves
 * populations, eqs. 3, 8 and 19 add none), so in a periodic or closed box
 * the FP64 mass changes only by rounding. With rel_tol > 0, the first
 * psm_get_stats after this call or after psm_set_equilibrium/psm_set_pdfs
 * records the mass as reference, and later calls return PSM_EDRIFT when
 * |mass - reference| > rel_tol |reference|. rel_tol = 0 turns it off.
 * PSM_EINVAL for a box with a pressure face or a face with a normal wall
 * velocity (they exchange mass). Host-only call. */
int psm_set_drift_check(psm_ctx* ctx, int box, double rel_tol);

/* Strict-slot mode (Sec. 3.1.1 keeps at most two solid fractions per cell).
 * Off (the default, or the environment variable PSM_STRICT_SLOTS unset or
 * not "1" at psm_create): a third overlap of a cell is dropped (the two
 * strongest stay) and counted by psm_get_stats. On: a step that meets such a
 * cell still runs the same way, and the next synchronising call returns
 * PSM_ECAPACITY; the context then refuses to step until psm_set_particles.
 * Overlaps met before the switch are forgotten. Synchronises. */
int psm_set_strict_slots(psm_ctx* ctx, int enable);

/* Sphere dynamics (Sec. 2.2.2) on the device, for collision-free spheres.
 * m = rho_p (4/3) pi r^3 and I = (2/5) m r^2 (fluid density 1); the total force
 * is the hydrodynamic force of the last executed step plus m * accel, the
 * torque is the hydrodynamic torque. */
enum psm_scheme {
    PSM_EULER = 0,   /* x += dt U; U += dt F/m; Omega += dt T/I */
    PSM_VERLET = 1   /* velocity Verlet, eqs. (15)-(16): U completed with the previous and the
                        new force (once a previous force exists), then x += dt U + dt^2 F/(2m) */
};

/* Density ratio rho_p > 0 and external acceleration accel (host double[3],
 * NULL = 0) of the spheres of box `box`. Defaults: 1 and 0. Synchronises. */
int psm_set_dynamics(psm_ctx* ctx, int box, double density_ratio, const double* accel);

/* Advance every sphere of every box by one update of `scheme` (psm_scheme)
 * with time step dt > 0, using the force and torque of the last executed
 * step; positions are wrapped into the box along periodic axes, and along an
 * axis with walls a centre leaving [r + 1, n_a - r - 1] is mirrored back with
 * its velocity component reversed (elastic contact; no sphere-sphere
 * contact is modelled). Then rebuild the per-tile
 * candidate lists on the device. Asynchronous: nothing is read back. If the
 * moved spheres put more than 64 candidates into a tile, the lists are cut
 * there (the step stays in bounds but its results are not valid) and the next
 * psm_get_forces / psm_get_stats / psm_get_particles returns PSM_ECAPACITY;
 * the context then refuses to step until psm_set_particles. psm_set_particles
 * restarts velocity Verlet (its first update has no previous force). */
int psm_integrate(psm_ctx* ctx, double dt, int scheme);

/* nsteps times (psm_step(ctx, 1) then psm_integrate(ctx, dt, scheme)), with
 * the host out of the loop: with graphs enabled (psm_set_graph), runs of 10
 * such pairs replay a captured HIP graph (recaptured when dt or scheme
 * change). Asynchronous; errors as psm_integrate. */
int psm_run(psm_ctx* ctx, int nsteps, double dt, int scheme);

/* Current positions x, velocities U and angular velocities omega of the
 * spheres of box `box` (host (n,3) each, any may be NULL). Synchronises;
 * reports a device-side list overflow as psm_integrate describes. */
int psm_get_particles(psm_ctx* ctx, int box, double* x, double* U, double* omega);

/* Launch options of the step kernel (bit flags). */
enum psm_launch_flags {
    PSM_LAUNCH_PERSISTENT = 1,  /* grid sized to the workgroups that fit on the chip at once; the
                                   workgroups on each of the 8 dies take the next tile of that die's
                                   eighth of the tile list from a counter the library zeroes before
                                   every step (else one workgroup per tile); same results bit for bit */
    PSM_LAUNCH_FILTER = 2       /* per wave and z, test each staged sphere against the rectangle of
                                   the wave's cells first; the per-cell mapping of Sec. 2.3.2 then
                                   visits only spheres that can reach them (same results) */
};

/* Launch shape of the step kernel: a tile of tx*ty threads (tx*ty == 256,
 * tx in {16,32,64,128,256}) handling tz cells each along z (tz in
 * {1,2,4,8,16,32}), and psm_launch_flags. Rebuilds the tile lists
 * (synchronises); invalidates captured graphs. On failure the previous
 * launch is restored. psm_get_launch: host outputs (flags may be NULL). */
int psm_set_launch(psm_ctx* ctx, int tx, int ty, int tz, int flags);
int psm_get_launch(psm_ctx* ctx, int* tx, int* ty, int* tz, int* flags);

/* Time every allowed launch shape and flag combination on this context with
 * HIP events (2 untimed + trial_steps timed steps each), then time the four
 * fastest twice more, interleaved, with 2 * trial_steps steps each; keep the
 * one with the smallest mean of those two and report it (host outputs, each
 * may be NULL). The trial steps advance and overwrite the PDF state: set the
 * state after tuning. Synchronises. best_ms: ms per step of the chosen launch
 * in the second round.
 * The pick is cached for the process, keyed by the GPU architecture, the
 * storage form, the mapping and, per box, its dimensions, walls and sphere
 * volume fraction (a power-of-two class); a context of a cached class gets
 * the cached launch and time without any trial (its state is then not
 * advanced). If the environment variable PSM_TUNE_CACHE names a file, its
 * entries are read at the first call and new picks are appended to it. */
int psm_autotune(psm_ctx* ctx, int trial_steps, int* tx, int* ty, int* tz, int* flags, double* best_ms);

/* Forget the autotune picks of this process (the file named by
 * PSM_TUNE_CACHE is not read again). Host-only call. */
int psm_clear_tune_cache(void);

/* Enable (1) / disable (0) HIP-graph replay of 10-step sequences in psm_step. */
int psm_set_graph(psm_ctx* ctx, int enable);

/* Kernel timing: when enabled, psm_step launches every step eagerly (no graph
 * replay) and records HIP events on the context's stream around every launch
 * of the step kernel.
 * psm_get_timing synchronises and returns the number of timed launches and
 * their summed duration in ms; psm_reset_timing clears both. The events come
 * from a pool of 128 pairs that the first psm_set_timing(ctx, 1) creates and
 * records once (it synchronises the stream then); every 128th timed launch
 * first waits for the earlier ones to finish and adds them up. */
int psm_set_timing(psm_ctx* ctx, int enable);
int psm_get_timing(psm_ctx* ctx, long long* launches, double* total_ms);
int psm_reset_timing(psm_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the mass and
 * momentum totals of psm_get_stats for a canonical FP64 field f (device
 * [19][ncells], the layout of psm_get_pdfs), without a context: out (device
 * double[4]) receives sum_x sum_q f, then sum_x sum_q f c_q (x, y, z).
 * Asynchronous on hip_stream, which must belong to the current device; it
 * calls no allocating routine. Its partial sums live in a library-owned
 * static device array of 128 KiB per GPU (kept until the process ends), so
 * ncells is at most 67,108,864 (PSM_EINVAL beyond); ncells = 0 gives zeros.
 * Calls that overlap on one GPU (different streams) race on that array. The
 * first call on a device looks the array up; make it outside stream capture. */
int psm_field_stats_noalloc(const double* f, long long ncells, double* out, void* hip_stream);

/* Bandwidth reference (the paper's SCALE/STREAM measurement, Sec. 4): copy
 * `bytes` (multiple of 16, at most 2^31 * 4 KiB) from src to dst (device,
 * 16-byte aligned, not overlapping) on hip_stream with a plain one-shot
 * streaming copy kernel. */
int psm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Bandwidth reference at the step's own access pattern (eq. 28 prices the
 * step by its PDF bytes; this measures the rate HBM serves those bytes in the
 * step's order): nrep launches of a kernel that walks every tile of every box
 * at the current launch shape and grid, pulls the 19 stored values of each
 * cell as psm_step does (shifted = 1: from x - c_q) or from the cell itself
 * (shifted = 0), and stores them unchanged at the cell in the grid psm_step
 * writes next, with no other arithmetic. The state psm_step reads is not
 * touched, so stepping may continue afterwards. Synchronises the context's
 * stream; *ms receives the average time of one launch (HIP events).
 * PSM_EINVAL for shifted other than 0/1, nrep < 1 or a NULL ms. */
int psm_pattern_copy(psm_ctx* ctx, int shifted, int nrep, double* ms);

/* Text of the last error on this thread ("" if none). Never NULL. */
const char* psm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PSM_H */
