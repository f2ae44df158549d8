/*
 * psm_oracle.c -- plain, slow FP64 CPU oracle of one PSM-LBM time step.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the correctness reference for the
 * GPU engine. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it. It shares no code, header, table or helper with
 * the GPU library, and the GPU library never calls it.
 *
 * Source: Kemmler, Rettinger, Ruede, Cuellar, Koestler, "Efficiency and
 * scalability of fully-resolved fluid-particle simulations on heterogeneous
 * CPU-GPU architectures" (arXiv 2303.11811).
 *   Sec. 2.1   lattice Boltzmann method, eqs. (1)-(8)
 *   Sec. 2.3   partially saturated cells method, eqs. (17)-(22)
 *   Sec. 2.3.2 particle mapping (linear approximation), eqs. (25)-(27)
 *   Sec. 2.2.2 particle integration, eqs. (15)-(16) (velocity Verlet), and
 *              the explicit Euler update of the moving-particle workload
 *
 * Scheme: push form exactly as eqs. (1)-(2) are written. The state f(x,t) is
 * the pre-collision PDF field. One step = map particles -> collide every cell
 * (eq. 17) and accumulate force/torque (eqs. 21-22) -> stream (eq. 2).
 *
 * Readings where the paper is silent or ambiguous:
 *   - D3Q19 velocity order and weights: the paper cites them only; the order
 *     below is the canonical I/O order of this project.
 *   - Forcing prefactor: eq. (8) is multiplied by (1 - 1/(2 tau)) (Guo et al.)
 *     so that the momentum input per step equals f_ext, matching the half-force
 *     velocity shift of eq. (7).
 *   - B > 1 (overlapping particles, Sec. 2.3): every slot fraction is divided
 *     by the cell's sum so that the total becomes exactly 1.
 *   - At most two particles per cell (Sec. 3.1.1): keep the two largest
 *     fractions (ties: smaller particle id), drop and count the rest, store
 *     the kept slots in ascending particle id.
 *   - B_i is the covered fraction itself (no tau-dependent weighting).
 *   - Cell (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2); all boxes are
 *     periodic and every displacement uses the minimum image.
 *   - Sub-division sampling (named in Sec. 2.3.2 as the alternative to the
 *     linear approximation): N^3 points at offsets (k+1/2)/N - 1/2 per axis,
 *     inclusion |s| <= r, evaluated without fused multiply-add.
 *   - No-slip walls (the paper's fluidized bed has them, Sec. 4; it does not
 *     name the scheme): half-way bounce-back at z = -1/2 and z = nz - 1/2 in
 *     cell-index coordinates, with the moving-wall term of Ladd for a wall
 *     velocity u_w (fluid density 1): a population f~_q leaving the fluid
 *     through the wall returns as f_qbar = f~_q - 6 w_q (c_q . u_w). A wall
 *     velocity with a normal component is a velocity inflow or outflow.
 *   - Side walls (x and y; the bed's four no-slip sides, Sec. 4): resting
 *     half-way bounce-back f_qbar = f~_q. A population that would leave
 *     through a side wall and a z face at once is bounced by the side wall.
 *   - Pressure outflow (named in Sec. 4, scheme not given): anti-bounce-back,
 *     f_qbar = -f~_q + 2 w_q (rho_w + 4.5 (c_q . u)^2 - 1.5 u.u), with u the
 *     boundary cell's post-collision velocity sum_q f~_q c_q of the same step.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared -o libpsm_oracle.so
 * The same source built with -fopenmp is a timing build: the collide-and-
 * stream loop of psmo_run is split over z-planes between threads, each thread
 * sums the force and torque of its own cells (in cell order) and the thread
 * sums are added in thread order. Built without OpenMP (the plain build every
 * test uses) there is one such sum, so it is the cell-order sum itself.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

/* D3Q19 velocities and weights (Sec. 2.1; weights of Qian et al.). */
static const int CQ[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};

static const double WQ[NQ] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Index of the inverse direction q-bar (c_qbar = -c_q), found by search. */
static int inverse_dir(int q)
{
    for (int p = 0; p < NQ; ++p)
        if (CQ[p][0] == -CQ[q][0] && CQ[p][1] == -CQ[q][1] && CQ[p][2] == -CQ[q][2])
            return p;
    return -1;
}

typedef struct {
    int nx, ny, nz;
    double tau;
    double fext[3];
    int mapping;   /* 0: linear approximation, 1: sub-division sampling */
    int nsub;      /* samples per axis for mapping == 1 */
    int walls_z;   /* bounded in z by faces at z = -1/2 and z = nz - 1/2 */
    double uwall[2][3];   /* velocities of the bottom and the top face (velocity faces) */
    int face_type[2];     /* 0: velocity (bounce-back), 1: pressure (anti-bounce-back) */
    double face_rho[2];   /* densities of pressure faces */
    int walls_x, walls_y; /* resting no-slip walls at x = -1/2, nx - 1/2 (and in y) */
} psmo_box;

typedef struct {
    int n;
    const double *x;     /* (n,3) centre, inside [0,L) */
    const double *r;     /* (n)   radius */
    const double *fr;    /* (n)   f(r) of eq. (26) */
    const double *U;     /* (n,3) translational velocity */
    const double *Om;    /* (n,3) angular velocity */
} psmo_particles;

/* ------------------------------------------------------------------ */
/* Threads of the collide-and-stream loop: the timing build (OpenMP) sets
 * and reports them (n <= 0 keeps the current count); the plain build has 1. */
int psmo_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Lattice export for the tests.                                        */
int psmo_lattice(int *c, double *w, int *qbar)
{
    for (int q = 0; q < NQ; ++q) {
        for (int a = 0; a < 3; ++a) c[3 * q + a] = CQ[q][a];
        w[q] = WQ[q];
        qbar[q] = inverse_dir(q);
    }
    return NQ;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3.2, eq. (27): V_a = integral over the unit square of
 * sqrt(r^2 - x^2 - y^2); eq. (26): f(r) = V_a - r + 1/2.              */
double psmo_Va(double r)
{
    double r2 = r * r;
    double s = sqrt(r2 - 0.5);
    double t1 = (1.0 / 12.0 - r2) * atan((0.5 * s) / (0.5 - r2));
    double t2 = (1.0 / 3.0) * s;
    double t3 = (r2 - 1.0 / 12.0) * atan(0.5 / s);
    double t4 = (4.0 / 3.0) * r * r2 * atan(0.25 / (r * s));
    return t1 + t2 + t3 - t4;
}

double psmo_fr(double r) { return psmo_Va(r) - r + 0.5; }

/* Minimum image of one displacement component into [-L/2, L/2). */
static double min_image(double d, double L)
{
    if (d >= 0.5 * L) return d - L;
    if (d < -0.5 * L) return d + L;
    return d;
}

static int wrap_index(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* Displacement from particle centre xp to the centre of cell (i,j,k). */
static void cell_displacement(const psmo_box *b, int i, int j, int k,
                              const double *xp, double d[3])
{
    d[0] = min_image((i + 0.5) - xp[0], (double)b->nx);
    d[1] = min_image((j + 0.5) - xp[1], (double)b->ny);
    d[2] = min_image((k + 0.5) - xp[2], (double)b->nz);
}

/* Overlap fraction of particle p with a cell whose centre sits at d from the
 * particle centre. Linear approximation: eps = f(r) - D with D = |d| - r
 * (eq. 26), overlap iff eps > 0, capped at 1. Sub-division sampling: fraction
 * of the nsub^3 sample points inside the sphere. Returns 0 for no overlap. */
static double overlap_fraction(const psmo_box *b, const double d[3], double r, double fr)
{
    if (b->mapping == 0) {
        double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double eps = fr - (dist - r);
        if (eps <= 0.0) return 0.0;
        return eps < 1.0 ? eps : 1.0;
    } else {
        int n = b->nsub;
        long inside = 0;
        double r2 = r * r;
        for (int kz = 0; kz < n; ++kz)
            for (int ky = 0; ky < n; ++ky)
                for (int kx = 0; kx < n; ++kx) {
                    double sx = d[0] + ((kx + 0.5) / n - 0.5);
                    double sy = d[1] + ((ky + 0.5) / n - 0.5);
                    double sz = d[2] + ((kz + 0.5) / n - 0.5);
                    double s2 = sx * sx + sy * sy + sz * sz;
                    if (s2 <= r2) ++inside;
                }
        return (double)inside / ((double)n * n * n);
    }
}

/* Two-slot list of one cell (Sec. 3.1.1: at most two fractions per cell). */
typedef struct {
    int ns;
    int pid[2];
    double B[2];
} slot2;

/* Candidate a is stronger than b: larger fraction, tie -> smaller id. */
static int stronger(double Ba, int pa, double Bb, int pb)
{
    return Ba > Bb || (Ba == Bb && pa < pb);
}

static void slot_insert(slot2 *s, int pid, double B, long long *overflow)
{
    if (s->ns < 2) {
        s->pid[s->ns] = pid;
        s->B[s->ns] = B;
        s->ns++;
        return;
    }
    int weak = stronger(s->B[0], s->pid[0], s->B[1], s->pid[1]) ? 1 : 0;
    if (stronger(B, pid, s->B[weak], s->pid[weak])) {
        s->pid[weak] = pid;
        s->B[weak] = B;
    }
    ++*overflow;
}

/* Ascending particle id, then B > 1 renormalisation (Sec. 2.3). */
static void slot_finish(slot2 *s)
{
    if (s->ns == 2 && s->pid[0] > s->pid[1]) {
        int tp = s->pid[0]; s->pid[0] = s->pid[1]; s->pid[1] = tp;
        double tb = s->B[0]; s->B[0] = s->B[1]; s->B[1] = tb;
    }
    if (s->ns == 2) {
        double sum = s->B[0] + s->B[1];
        if (sum > 1.0) {
            s->B[0] = s->B[0] / sum;
            s->B[1] = s->B[1] / sum;
        }
    }
}

/* Mapping of all particles onto the box: for each particle in order, every
 * cell of its (wrapped) bounding box [x_p - (r+1), x_p + (r+1)].          */
static void map_all(const psmo_box *b, const psmo_particles *P, slot2 *slots,
                    long long *overflow)
{
    long N = (long)b->nx * b->ny * b->nz;
    for (long n = 0; n < N; ++n) slots[n].ns = 0;
    for (int p = 0; p < P->n; ++p) {
        const double *xp = P->x + 3 * p;
        double r = P->r[p];
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = (int)floor(xp[a] - (r + 1.0));
            hi[a] = (int)floor(xp[a] + (r + 1.0));
        }
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
            for (int jj = lo[1]; jj <= hi[1]; ++jj)
                for (int ii = lo[0]; ii <= hi[0]; ++ii) {
                    int i = wrap_index(ii, b->nx), j = wrap_index(jj, b->ny), k = wrap_index(kk, b->nz);
                    double d[3];
                    cell_displacement(b, i, j, k, xp, d);
                    double B = overlap_fraction(b, d, r, P->fr[p]);
                    if (B > 0.0)
                        slot_insert(&slots[i + (long)b->nx * (j + (long)b->ny * k)], p, B, overflow);
                }
    }
    for (long n = 0; n < N; ++n) slot_finish(&slots[n]);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.1, eq. (5): incompressible equilibrium with rho_0 = 1, c_s^2 = 1/3. */
static double equilibrium(int q, double rho, const double V[3])
{
    double cv = CQ[q][0] * V[0] + CQ[q][1] * V[1] + CQ[q][2] * V[2];
    double vv = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    return WQ[q] * (rho + 3.0 * cv + 4.5 * cv * cv - 1.5 * vv);
}

/* Eqs. (6)-(7): density and half-force-shifted velocity of a cell. */
static void moments(const psmo_box *b, const double f[NQ], double *rho, double U[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < NQ; ++q) {
        r += f[q];
        for (int a = 0; a < 3; ++a) j[a] += f[q] * CQ[q][a];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) U[a] = j[a] + 0.5 * b->fext[a];
}

static void cross(const double a[3], const double c[3], double out[3])
{
    out[0] = a[1] * c[2] - a[2] * c[1];
    out[1] = a[2] * c[0] - a[0] * c[2];
    out[2] = a[0] * c[1] - a[1] * c[0];
}

/* Collision of one cell, eqs. (3), (8), (17)-(22).
 * f:  pre-collision PDFs; ft: post-collision PDFs (output).
 * ns slots with particle ids pid[] and fractions B[] (already renormalised).
 * g (ns x 3, optional): sum_q C^solid_{q,s} c_qbar of each slot, the per-cell
 * factor of eqs. (21)-(22). d (ns x 3, optional): cell-centre lever arm.    */
static void collide_cell(const psmo_box *b, int i, int j, int k, const double f[NQ],
                         int ns, const int *pid, const double *Bs,
                         const psmo_particles *P, double ft[NQ], double *g, double *dout)
{
    double rho, U[3];
    moments(b, f, &rho, U);
    double tau = b->tau;

    double Btot = 0.0;
    for (int s = 0; s < ns; ++s) Btot += Bs[s];

    /* Solid collision operators per slot, eq. (19); particle velocity at the
     * cell centre, eq. (20). */
    double Csol[2][NQ];
    double dvec[2][3];
    for (int s = 0; s < ns; ++s) {
        int p = pid[s];
        cell_displacement(b, i, j, k, P->x + 3 * p, dvec[s]);
        double w_x_d[3], V[3];
        cross(P->Om + 3 * p, dvec[s], w_x_d);
        for (int a = 0; a < 3; ++a) V[a] = P->U[3 * p + a] + w_x_d[a];
        for (int q = 0; q < NQ; ++q) {
            int qb = inverse_dir(q);
            Csol[s][q] = (f[qb] - equilibrium(qb, rho, U)) - (f[q] - equilibrium(q, rho, V));
        }
    }

    double pref = 1.0 - 1.0 / (2.0 * tau);
    for (int q = 0; q < NQ; ++q) {
        /* eq. (3) with Delta t = 1 */
        double Csrt = (equilibrium(q, rho, U) - f[q]) / tau;
        /* eq. (8), Guo prefactor (1 - 1/(2 tau)), c_s^2 = 1/3, c_s^4 = 1/9 */
        double cu = CQ[q][0] * U[0] + CQ[q][1] * U[1] + CQ[q][2] * U[2];
        double Fq = 0.0;
        for (int a = 0; a < 3; ++a)
            Fq += (3.0 * (CQ[q][a] - U[a]) + 9.0 * cu * CQ[q][a]) * b->fext[a];
        Fq = pref * WQ[q] * Fq;
        /* eqs. (17)-(18) */
        double sol = 0.0;
        for (int s = 0; s < ns; ++s) sol += Bs[s] * Csol[s][q];
        ft[q] = f[q] + (1.0 - Btot) * Csrt + sol + (1.0 - Btot) * Fq;
    }

    /* Per-slot factor of eqs. (21)-(22): sum_q C^solid_q c_qbar = -sum_q C^solid_q c_q. */
    for (int s = 0; s < ns; ++s) {
        double gs[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < NQ; ++q)
            for (int a = 0; a < 3; ++a) gs[a] -= Csol[s][q] * CQ[q][a];
        if (g)
            for (int a = 0; a < 3; ++a) g[3 * s + a] = gs[a];
        if (dout)
            for (int a = 0; a < 3; ++a) dout[3 * s + a] = dvec[s][a];
    }
}

/* ------------------------------------------------------------------ */
/* Public oracle entry points (called from Python through ctypes).      */

static psmo_particles make_particles(int n, const double *x, const double *r, const double *fr,
                                     const double *U, const double *Om)
{
    psmo_particles P = {n, x, r, fr, U, Om};
    return P;
}

/* Equilibrium initialisation f_q = E_q(rho, u) (eq. 5). rho may be NULL (=1).
 * u is [3][N]. f is [19][N]. */
void psmo_equilibrium_field(const psmo_box *b, const double *rho, const double *u, double *f)
{
    long N = (long)b->nx * b->ny * b->nz;
    for (long n = 0; n < N; ++n) {
        double V[3] = {u[n], u[N + n], u[2 * N + n]};
        double r = rho ? rho[n] : 1.0;
        for (int q = 0; q < NQ; ++q) f[q * N + n] = equilibrium(q, r, V);
    }
}

/* Density and velocity (eqs. 6-7) of a [19][N] field. */
void psmo_macroscopic(const psmo_box *b, const double *f, double *rho, double *u)
{
    long N = (long)b->nx * b->ny * b->nz;
    for (long n = 0; n < N; ++n) {
        double fc[NQ], r, U[3];
        for (int q = 0; q < NQ; ++q) fc[q] = f[q * N + n];
        moments(b, fc, &r, U);
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[a * N + n] = U[a];
    }
}

/* Mapping only: B [2][N] and pid [2][N] (-1 = empty slot). Returns the number
 * of dropped (cell, particle) overlaps. */
long long psmo_map(const psmo_box *b, int np, const double *x, const double *r, const double *fr,
                   double *B, int *pid)
{
    long N = (long)b->nx * b->ny * b->nz;
    psmo_particles P = make_particles(np, x, r, fr, NULL, NULL);
    slot2 *slots = (slot2 *)malloc(sizeof(slot2) * (size_t)N);
    long long overflow = 0;
    map_all(b, &P, slots, &overflow);
    for (long n = 0; n < N; ++n) {
        for (int s = 0; s < 2; ++s) {
            B[s * N + n] = s < slots[n].ns ? slots[n].B[s] : 0.0;
            pid[s * N + n] = s < slots[n].ns ? slots[n].pid[s] : -1;
        }
    }
    free(slots);
    return overflow;
}

/* Slots of a single cell by brute force over every particle (same rules as
 * psmo_map, used to check sampled cells of large boxes). Returns ns. */
int psmo_map_cell(const psmo_box *b, int i, int j, int k, int np, const double *x,
                  const double *r, const double *fr, int *pid2, double *B2, long long *overflow)
{
    slot2 s;
    s.ns = 0;
    long long ov = 0;
    for (int p = 0; p < np; ++p) {
        double d[3];
        cell_displacement(b, i, j, k, x + 3 * p, d);
        double B = overlap_fraction(b, d, r[p], fr[p]);
        if (B > 0.0) slot_insert(&s, p, B, &ov);
    }
    slot_finish(&s);
    for (int t = 0; t < 2; ++t) {
        pid2[t] = t < s.ns ? s.pid[t] : -1;
        B2[t] = t < s.ns ? s.B[t] : 0.0;
    }
    if (overflow) *overflow = ov;
    return s.ns;
}

/* Collision of one cell with explicit slots (for sampled checks).
 * g (ns x 3) receives sum_q C^solid c_qbar per slot. */
void psmo_collide_cell(const psmo_box *b, int i, int j, int k, const double *f19, int ns,
                       const int *pid, const double *Bs, int np, const double *x,
                       const double *U, const double *Om, double *ft19, double *g)
{
    psmo_particles P = make_particles(np, x, NULL, NULL, U, Om);
    collide_cell(b, i, j, k, f19, ns, pid, Bs, &P, ft19, g, NULL);
}

/* nsteps full time steps on f ([19][N], pre-collision, in/out).
 * Outputs of the LAST step: F, T (np,3) by eqs. (21)-(22) accumulated in cell
 * order; Ascale (np) = sum over cells and slots of B_s |g_s| (the magnitude
 * scale of the force sum); B/pid [2][N] slots of the last mapping (optional).
 * Returns the total slot overflow count of the last step's mapping. */
long long psmo_run(const psmo_box *b, int nsteps, int np, const double *x, const double *r,
                   const double *fr, const double *U, const double *Om, double *f,
                   double *F, double *T, double *Ascale, double *Bout, int *pidout)
{
    int nx = b->nx, ny = b->ny, nz = b->nz;
    long N = (long)nx * ny * nz;
    psmo_particles P = make_particles(np, x, r, fr, U, Om);
    slot2 *slots = (slot2 *)malloc(sizeof(slot2) * (size_t)N);
    double *fnew = (double *)malloc(sizeof(double) * (size_t)NQ * (size_t)N);
    long long overflow = 0;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    /* per-thread force, torque and force-scale sums: [thread][np][3], [thread][np] */
    size_t np1 = np > 0 ? (size_t)np : 1;
    double *Fth = (double *)malloc(sizeof(double) * 3 * np1 * (size_t)nth);
    double *Tth = (double *)malloc(sizeof(double) * 3 * np1 * (size_t)nth);
    double *Ath = (double *)malloc(sizeof(double) * np1 * (size_t)nth);

    for (int step = 0; step < nsteps; ++step) {
        overflow = 0;
        map_all(b, &P, slots, &overflow);
        for (size_t e = 0; e < 3 * np1 * (size_t)nth; ++e) { Fth[e] = 0.0; Tth[e] = 0.0; }
        for (size_t e = 0; e < np1 * (size_t)nth; ++e) Ath[e] = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int k = 0; k < nz; ++k) {
            int th = 0;
#ifdef _OPENMP
            th = omp_get_thread_num();
#endif
            double *Fs = Fth + 3 * np1 * (size_t)th, *Ts = Tth + 3 * np1 * (size_t)th;
            double *As = Ascale ? Ath + np1 * (size_t)th : NULL;
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    long n = i + (long)nx * (j + (long)ny * k);
                    double fc[NQ], ft[NQ], g[6], d[6];
                    for (int q = 0; q < NQ; ++q) fc[q] = f[q * N + n];
                    slot2 *s = &slots[n];
                    collide_cell(b, i, j, k, fc, s->ns, s->pid, s->B, &P, ft, g, d);
                    /* eqs. (21)-(22) with Delta x = Delta t = 1 */
                    for (int t = 0; t < s->ns; ++t) {
                        int p = s->pid[t];
                        double Bg[3], tq[3];
                        for (int a = 0; a < 3; ++a) Bg[a] = s->B[t] * g[3 * t + a];
                        cross(d + 3 * t, Bg, tq);
                        for (int a = 0; a < 3; ++a) {
                            Fs[3 * p + a] += Bg[a];
                            Ts[3 * p + a] += tq[a];
                        }
                        if (As)
                            As[p] += s->B[t] * sqrt(g[3 * t] * g[3 * t] + g[3 * t + 1] * g[3 * t + 1] +
                                                    g[3 * t + 2] * g[3 * t + 2]);
                    }
                    /* eq. (2): f_q(x + c_q, t + 1) = ft_q(x, t) */
                    for (int q = 0; q < NQ; ++q) {
                        int ii = i + CQ[q][0], jj = j + CQ[q][1], kk = k + CQ[q][2];
                        if ((b->walls_x && (ii < 0 || ii >= nx)) || (b->walls_y && (jj < 0 || jj >= ny))) {
                            /* resting side wall: half-way bounce-back */
                            fnew[inverse_dir(q) * N + n] = ft[q];
                            continue;
                        }
                        if (b->walls_z && (kk < 0 || kk >= nz)) {
                            int face = kk < 0 ? 0 : 1;
                            if (b->face_type[face] == 1) {
                                /* anti-bounce-back with the cell's post-collision velocity */
                                double u[3] = {0.0, 0.0, 0.0};
                                for (int p = 0; p < NQ; ++p)
                                    for (int a = 0; a < 3; ++a) u[a] += ft[p] * CQ[p][a];
                                double cu = CQ[q][0] * u[0] + CQ[q][1] * u[1] + CQ[q][2] * u[2];
                                double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                                fnew[inverse_dir(q) * N + n] =
                                    -ft[q] + 2.0 * WQ[q] * (b->face_rho[face] + 4.5 * cu * cu - 1.5 * uu);
                                continue;
                            }
                            /* half-way bounce-back, moving-wall term for the wall crossed */
                            const double *uw = b->uwall[face];
                            double cu = CQ[q][0] * uw[0] + CQ[q][1] * uw[1] + CQ[q][2] * uw[2];
                            fnew[inverse_dir(q) * N + n] = ft[q] - 6.0 * WQ[q] * cu;
                            continue;
                        }
                        ii = wrap_index(ii, nx);
                        jj = wrap_index(jj, ny);
                        kk = wrap_index(kk, nz);
                        fnew[q * N + ii + (long)nx * (jj + (long)ny * kk)] = ft[q];
                    }
                }
        }
        for (int p = 0; p < np; ++p) {
            for (int a = 0; a < 3; ++a) {
                double fs = 0.0, ts = 0.0;
                for (int th = 0; th < nth; ++th) {
                    fs += Fth[3 * np1 * (size_t)th + 3 * p + a];
                    ts += Tth[3 * np1 * (size_t)th + 3 * p + a];
                }
                F[3 * p + a] = fs;
                T[3 * p + a] = ts;
            }
            if (Ascale) {
                double as = 0.0;
                for (int th = 0; th < nth; ++th) as += Ath[np1 * (size_t)th + p];
                Ascale[p] = as;
            }
        }
        memcpy(f, fnew, sizeof(double) * (size_t)NQ * (size_t)N);
    }
    free(Fth);
    free(Tth);
    free(Ath);

    if (Bout && pidout) {
        for (long n = 0; n < N; ++n)
            for (int t = 0; t < 2; ++t) {
                Bout[t * N + n] = t < slots[n].ns ? slots[n].B[t] : 0.0;
                pidout[t * N + n] = t < slots[n].ns ? slots[n].pid[t] : -1;
            }
    }
    free(fnew);
    free(slots);
    return overflow;
}

/* ------------------------------------------------------------------ */
/* Particle integration (Sec. 2.2.2) for spheres without collisions.    */
/*
 * Mass and moment of inertia of a homogeneous sphere of radius r and density
 * ratio rho_p (fluid density 1): m = rho_p (4/3) pi r^3, I = (2/5) m r^2.
 * The total force is the hydrodynamic force plus m * accel (an external
 * acceleration such as gravity minus buoyancy); the torque is hydrodynamic.
 *
 * scheme 0, explicit Euler:   x += dt U;  U += dt F/m;  Om += dt T/I.
 * scheme 1, velocity Verlet of eqs. (15)-(16), called once after each fluid
 * step with that step's force F (taken at the positions x it used):
 *   if have_prev:  U  += dt/(2m) (F_prev + F),  Om += dt/(2I) (T_prev + T)
 *   then           x  += dt U + dt^2/(2m) F,    F_prev = F, T_prev = T.
 * Positions are wrapped into [0, L) afterwards along periodic axes; along an
 * axis with walls (walls[a] != 0) a centre that leaves [r + 1, L - r - 1] is
 * mirrored back and its velocity component reversed (an elastic contact that
 * keeps the one-cell gap the solid-fraction mapping needs; the paper's DEM
 * contact with the bounding planes is out of scope). Arrays (n,3) row-major,
 * updated in place. */
static double wrap_coord(double v, double L)
{
    double w = fmod(v, L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    return w;
}

void psmo_integrate(int n, int scheme, double dt, double rho_p, const double *accel, const double *Lbox,
                    const int *walls, const double *r, double *x, double *U, double *Om, const double *F,
                    const double *T, double *Fprev, double *Tprev, int have_prev)
{
    const double pi = 3.14159265358979323846;
    for (int p = 0; p < n; ++p) {
        double m = rho_p * (4.0 / 3.0) * pi * r[p] * r[p] * r[p];
        double I = 0.4 * m * r[p] * r[p];
        double Ft[3], Tt[3];
        for (int a = 0; a < 3; ++a) {
            Ft[a] = F[3 * p + a] + m * accel[a];
            Tt[a] = T[3 * p + a];
        }
        if (scheme == 0) {
            for (int a = 0; a < 3; ++a) {
                x[3 * p + a] += dt * U[3 * p + a];
                U[3 * p + a] += dt * Ft[a] / m;
                Om[3 * p + a] += dt * Tt[a] / I;
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                if (have_prev) {
                    U[3 * p + a] += dt / (2.0 * m) * (Fprev[3 * p + a] + Ft[a]);
                    Om[3 * p + a] += dt / (2.0 * I) * (Tprev[3 * p + a] + Tt[a]);
                }
                x[3 * p + a] += dt * U[3 * p + a] + dt * dt / (2.0 * m) * Ft[a];
                Fprev[3 * p + a] = Ft[a];
                Tprev[3 * p + a] = Tt[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            if (!walls[a]) {
                x[3 * p + a] = wrap_coord(x[3 * p + a], Lbox[a]);
                continue;
            }
            /* elastic contact with the walls of this axis, one cell before
               the sphere reaches them: mirror the centre back into
               [r + 1, L - r - 1] and reverse the normal velocity */
            double lo = r[p] + 1.0, hi = Lbox[a] - r[p] - 1.0;
            if (x[3 * p + a] < lo) {
                x[3 * p + a] = 2.0 * lo - x[3 * p + a];
                U[3 * p + a] = -U[3 * p + a];
            } else if (x[3 * p + a] > hi) {
                x[3 * p + a] = 2.0 * hi - x[3 * p + a];
                U[3 * p + a] = -U[3 * p + a];
            }
        }
    }
}
