/*
 * FP64 CPU oracle for the moment-only, high-order thread-safe lattice
 * Boltzmann update (Montessori et al., "High-order thread-safe lattice
 * Boltzmann model for HPC turbulent flow simulations", arXiv:2401.17074).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously
 * correct definition the GPU path is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * Every population is evaluated from the explicit Hermite-tensor formulas
 * (Section 2.2) in double precision; moments are plain sums over the 27
 * velocities.  Derivatives (for the adjoint and tangent checks) are taken by
 * the complex-step method on the very same formulas.
 *
 * State layout (all arrays double, SoA, x fastest):
 *   st[q*N + n], n = x + nx*(y + ny*z), q = 0 rho, 1..3 u, 4..9 Pi^neq
 *   with Pi ordered xx, yy, zz, xy, xz, yz.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 27 /* the most velocities of a supported lattice (D3Q27) */
static const double CS2 = 1.0 / 3.0; /* lattice sound speed squared, Eq. (lbequil) */

/* ------------------------------------------------------------------ */
/* Lattices (Section 2.1, the D3Q27 figure; D2Q9 is its two-dimensional
 * counterpart named in Section 2.2).  The weights are not printed in the
 * paper; they are the tensor products of the one-dimensional three-point
 * Gauss-Hermite weights W(0) = 2/3, W(+-1) = 1/6, the unique sets giving
 * the isotropy the text relies on (sum w c c = cs2 delta up to the
 * highest-order moment, e.g. sum w cx^2 cy^2 cz^2 = cs2^3 in 3D).  D2Q9
 * velocities are stored as 3-vectors with c_z = 0.                         */
typedef struct {
    int q, d;        /* number of velocities, spatial dimensions */
    int c[NQ][3];
    double w[NQ];
    int opp[NQ];
} lattice_t;

static lattice_t LAT27, LAT9, LAT19;
static const int PI_IDX[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};

static void build_lattice(lattice_t *L, int d)
{
    int i = 0;
    for (int cx = -1; cx <= 1; cx++)
        for (int cy = -1; cy <= 1; cy++)
            for (int cz = (d == 3 ? -1 : 0); cz <= (d == 3 ? 1 : 0); cz++) {
                L->c[i][0] = cx;
                L->c[i][1] = cy;
                L->c[i][2] = cz;
                double w = 1.0;
                for (int a = 0; a < d; a++) w *= (L->c[i][a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
                L->w[i] = w;
                i++;
            }
    L->q = i;
    L->d = d;
    for (int a = 0; a < L->q; a++)
        for (int b = 0; b < L->q; b++)
            if (L->c[a][0] == -L->c[b][0] && L->c[a][1] == -L->c[b][1] && L->c[a][2] == -L->c[b][2]) L->opp[a] = b;
}

/* D3Q19: the rest, face and edge velocities of D3Q27 (no corners), with
 * the unique shell weights for sum w = 1, sum w cx^2 = cs2 and
 * sum w cx^2 cy^2 = cs2^2: 1/3, 1/18, 1/36.                                 */
static void build_d3q19(lattice_t *L)
{
    const double ws[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    int i = 0;
    for (int cx = -1; cx <= 1; cx++)
        for (int cy = -1; cy <= 1; cy++)
            for (int cz = -1; cz <= 1; cz++) {
                const int shell = abs(cx) + abs(cy) + abs(cz);
                if (shell == 3) continue;
                L->c[i][0] = cx;
                L->c[i][1] = cy;
                L->c[i][2] = cz;
                L->w[i] = ws[shell];
                i++;
            }
    L->q = i;
    L->d = 3;
    for (int a = 0; a < L->q; a++)
        for (int b = 0; b < L->q; b++)
            if (L->c[a][0] == -L->c[b][0] && L->c[a][1] == -L->c[b][1] && L->c[a][2] == -L->c[b][2]) L->opp[a] = b;
}

static void lattice_init(void)
{
    static int done = 0;
    if (done) return;
    build_lattice(&LAT27, 3);
    build_lattice(&LAT9, 2);
    build_d3q19(&LAT19);
    done = 1;
}

static const lattice_t *lattice_of(int id) { return id == 9 ? &LAT9 : (id == 19 ? &LAT19 : &LAT27); }

static double hermite1(const lattice_t *L, int i, int a) { return (double)L->c[i][a]; }

static double hermite2(const lattice_t *L, int i, int a, int b)
{
    return (double)(L->c[i][a] * L->c[i][b]) - CS2 * (a == b);
}

static double hermite3(const lattice_t *L, int i, int a, int b, int g)
{
    const int *c = L->c[i];
    return (double)(c[a] * c[b] * c[g]) - CS2 * (c[g] * (a == b) + c[a] * (b == g) + c[b] * (a == g));
}

/* ------------------------------------------------------------------ */
/* Grid, faces and node classes.                                       */
enum { FACE_PERIODIC = 0, FACE_WALL = 1, FACE_INLET = 2, FACE_OUTLET = 3 };
enum { NODE_FLUID = 0, NODE_SOLID = 1, NODE_GHOST = 2 };

typedef struct {
    int nx, ny, nz;
    int face[6]; /* -x, +x, -y, +y, -z, +z */
    double tau;
    double force[3]; /* uniform body acceleration (used when no field is given) */
    double inlet_u[3];
    double inlet_center[2]; /* transverse coordinates of the inlet disc centre */
    double inlet_radius;
    double inlet_noise; /* relative amplitude of the inlet perturbation */
    uint64_t seed;
    int order; /* Hermite order of the reconstruction: 3 (Section 2.2) or 2 (Eq. (fullstrcoll)) */
    int noise_kind; /* inlet perturbation: 0 uniform in [-1, 1), 1 standard Gaussian (Section 3.2) */
    const double *tau_z; /* relaxation time of each z plane (the jet's outlet sponge), or NULL: tau */
    int lattice; /* 27 (or 0): D3Q27; 19: D3Q19; 9: D2Q9 on an nz = 1 grid with periodic z faces */
} or_grid;

static const lattice_t *lat(const or_grid *G) { return lattice_of(G->lattice); }

static int dim(const or_grid *G, int d) { return d == 0 ? G->nx : (d == 1 ? G->ny : G->nz); }
static int is_ghost_face(int k) { return k == FACE_INLET || k == FACE_OUTLET; }

static void node_coords(const or_grid *G, long n, int x[3])
{
    x[0] = (int)(n % G->nx);
    x[1] = (int)((n / G->nx) % G->ny);
    x[2] = (int)(n / ((long)G->nx * G->ny));
}

/* Relaxation frequency omega = 1/tau of node n: the plane's entry of the
 * sponge profile when one is given (Section 3.2), else the global tau.      */
static double omega_at(const or_grid *G, long n)
{
    if (!G->tau_z) return 1.0 / G->tau;
    return 1.0 / G->tau_z[n / ((long)G->nx * G->ny)];
}

static long node_index(const or_grid *G, const int x[3])
{
    return (long)x[0] + (long)G->nx * ((long)x[1] + (long)G->ny * x[2]);
}

/* A node on a wall face layer is solid (walls win over ghosts); a node on
 * an inflow/outflow face layer is a ghost; every other node is fluid.       */
static int node_kind_xyz(const or_grid *G, const int x[3])
{
    int ghost = 0;
    for (int d = 0; d < 3; d++) {
        int lo = x[d] == 0, hi = x[d] == dim(G, d) - 1;
        if ((lo && G->face[2 * d] == FACE_WALL) || (hi && G->face[2 * d + 1] == FACE_WALL)) return NODE_SOLID;
        if ((lo && is_ghost_face(G->face[2 * d])) || (hi && is_ghost_face(G->face[2 * d + 1]))) ghost = 1;
    }
    return ghost ? NODE_GHOST : NODE_FLUID;
}

static int node_kind(const or_grid *G, long n)
{
    int x[3];
    node_coords(G, n, x);
    return node_kind_xyz(G, x);
}

static int grid_has_ghosts(const or_grid *G)
{
    for (int f = 0; f < 6; f++)
        if (is_ghost_face(G->face[f])) return 1;
    return 0;
}

/* Index of the upstream node x - c_i (periodic axes wrap); -1 if it is solid. */
static long upstream(const or_grid *G, const int x[3], int i)
{
    int y[3];
    for (int d = 0; d < 3; d++) {
        int n = dim(G, d);
        y[d] = x[d] - lat(G)->c[i][d];
        if (G->face[2 * d] == FACE_PERIODIC) y[d] = ((y[d] % n) + n) % n;
        if (y[d] < 0 || y[d] >= n) return -2; /* cannot happen for a fluid node */
    }
    if (node_kind_xyz(G, y) == NODE_SOLID) return -1;
    return node_index(G, y);
}

/* Nearest interior node of a ghost node: clamp along each ghost axis. */
static void interior_neighbour(const or_grid *G, const int x[3], int xf[3])
{
    for (int d = 0; d < 3; d++) {
        xf[d] = x[d];
        if (x[d] == 0 && is_ghost_face(G->face[2 * d])) xf[d] = 1;
        if (x[d] == dim(G, d) - 1 && is_ghost_face(G->face[2 * d + 1])) xf[d] = dim(G, d) - 2;
    }
}

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the k-th output (k >= 1) of
 * the generator seeded with `seed` is mix(seed + k * 0x9e3779b97f4a7c15).   */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* Uniform variate in [-1, 1) for (level t, node n, component a): the top 24
 * bits of output k = 1 + 3 (t N + n) + a.  Exact in binary32 and binary64.  */
static double inlet_xi(uint64_t seed, long t, long n, long N, int a)
{
    uint64_t k = 1ULL + 3ULL * ((uint64_t)t * (uint64_t)N + (uint64_t)n) + (uint64_t)a;
    uint64_t h = splitmix64_at(seed, k);
    return ldexp((double)(h >> 40), -24) * 2.0 - 1.0;
}

/* Standard Gaussian variate for (level t, node n, component a) by the
 * Box-Muller transform (Box and Muller 1958) of two uniforms drawn from
 * outputs k1 = 1 + 6 (t N + n) + 2 a and k1 + 1 of the same stream:
 *   v1 = (top 24 bits of output k1 + 1) 2^-24   in (0, 1]
 *   v2 = (top 24 bits of output k1 + 1 + 1) 2^-24 in [0, 1)
 *   xi = sqrt(-2 ln v1) cos(2 pi v2).                                        */
static double inlet_gauss(uint64_t seed, long t, long n, long N, int a)
{
    uint64_t k = 1ULL + 6ULL * ((uint64_t)t * (uint64_t)N + (uint64_t)n) + 2ULL * (uint64_t)a;
    double v1 = ldexp((double)((splitmix64_at(seed, k) >> 40) + 1), -24);
    double v2 = ldexp((double)(splitmix64_at(seed, k + 1) >> 40), -24);
    return sqrt(-2.0 * log(v1)) * cos(6.283185307179586476925286766559 * v2);
}

/* Imposed velocity of an inlet-disc ghost node at level t (top hat plus the
 * seeded perturbation); returns 0 if the node is not on an inlet disc.      */
static int inlet_velocity(const or_grid *G, const int x[3], long n, long t, double ub[3])
{
    const long N = (long)G->nx * G->ny * G->nz;
    for (int f = 0; f < 6; f++) {
        if (G->face[f] != FACE_INLET) continue;
        int d = f / 2;
        int layer = (f % 2 == 0) ? 0 : dim(G, d) - 1;
        if (x[d] != layer) continue;
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        if (d1 > d2) { int tmp = d1; d1 = d2; d2 = tmp; }
        double r1 = x[d1] - G->inlet_center[0], r2 = x[d2] - G->inlet_center[1];
        if (r1 * r1 + r2 * r2 > G->inlet_radius * G->inlet_radius) continue;
        double mag = sqrt(G->inlet_u[0] * G->inlet_u[0] + G->inlet_u[1] * G->inlet_u[1] +
                          G->inlet_u[2] * G->inlet_u[2]);
        for (int a = 0; a < 3; a++) {
            ub[a] = G->inlet_u[a];
            if (a < lat(G)->d)
                ub[a] += G->inlet_noise * mag *
                         (G->noise_kind == 1 ? inlet_gauss(G->seed, t, n, N, a) : inlet_xi(G->seed, t, n, N, a));
        }
        return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The arithmetic, instantiated for double and for double complex.     */
#define R double
#define FN(name) name##_r
#include "tslb_core.inc"
#undef R
#undef FN

#define R double complex
#define FN(name) name##_c
#include "tslb_core.inc"
#undef R
#undef FN

static const double CSTEP = 1e-30; /* complex-step size */

/* ------------------------------------------------------------------ */
/* IEEE 754 round-to-nearest-even into a binary format with `frac` stored
 * fraction bits, minimum normal exponent `emin` and largest finite `maxv`.
 * Subnormals use the fixed quantum 2^(emin - frac); overflow gives inf.     */
static double round_binary(double x, int frac, int emin, double maxv)
{
    if (x == 0.0 || !isfinite(x)) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e); /* ax = m 2^e, m in [0.5, 1): floor(log2 ax) = e - 1 */
    int E = e - 1;
    if (E < emin) E = emin;
    double q = ldexp(1.0, E - frac);
    double r = nearbyint(ax / q) * q; /* default rounding mode: ties to even */
    if (r > maxv) r = INFINITY;
    return copysign(r, x);
}

double or_round_fp16(double x) { return round_binary(x, 10, -14, 65504.0); }
double or_round_bf16(double x) { return round_binary(x, 7, -126, ldexp(255.0, 120)); }

/* ================================================================== */
/* Exported API (ctypes).                                              */

/* Velocities (3 ints each), weights and opposites of lattice 27 or 9;
 * returns the number of velocities.                                         */
int or_lattice(int lattice, int *c, double *w, int *opp)
{
    lattice_init();
    const lattice_t *L = lattice_of(lattice);
    for (int i = 0; i < L->q; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = L->c[i][a];
        w[i] = L->w[i];
        opp[i] = L->opp[i];
    }
    return L->q;
}

/* Hermite tensor component of order `order` (0..3) at velocity i. */
double or_hermite(int lattice, int i, int order, int a, int b, int g)
{
    lattice_init();
    const lattice_t *L = lattice_of(lattice);
    switch (order) {
    case 0: return 1.0;
    case 1: return hermite1(L, i, a);
    case 2: return hermite2(L, i, a, b);
    case 3: return hermite3(L, i, a, b, g);
    }
    return NAN;
}

double or_feq(int lattice, int i, double rho, const double *u, int order)
{
    lattice_init();
    return feq_r(lattice_of(lattice), i, rho, u, order);
}

double or_fneq(int lattice, int i, const double *pi6, const double *u, int order)
{
    lattice_init();
    double pi[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) pi[a][b] = pi6[PI_IDX[a][b]];
    return fneq_r(lattice_of(lattice), i, pi, u, order);
}

double or_fpost(int lattice, int i, const double *m, const double *g, double omega, int order)
{
    lattice_init();
    return fpost_r(lattice_of(lattice), i, m, g, omega, order);
}

void or_moments(int lattice, const double *f, double *m)
{
    lattice_init();
    moments_r(lattice_of(lattice), f, m);
}

int or_node_kind(const or_grid *G, long n) { return node_kind(G, n); }

void or_node_kinds(const or_grid *G, signed char *out)
{
    const long N = (long)G->nx * G->ny * G->nz;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; n++) out[n] = (signed char)node_kind(G, n);
}

void or_ghost_fill(const or_grid *G, double *st, long t)
{
    lattice_init();
    ghost_fill_r(G, st, t);
}

/* One step: out <- update(in) at level t -> t+1 (ghosts of out refilled). */
void or_step(const or_grid *G, const double *in, double *out, const double *gf, long t)
{
    lattice_init();
    step_r(G, in, out, gf, t);
}

/* Storage rounding emulation: the stored quantities (rho - 1) s0, u s1 and
 * Pi s2 are rounded to binary16 (kind 1) or bfloat16 (kind 2).             */
void or_round_storage(const or_grid *G, double *st, int kind, const double *scale)
{
    const long N = (long)G->nx * G->ny * G->nz;
    double (*rnd)(double) = kind == 1 ? or_round_fp16 : or_round_bf16;
    for (long n = 0; n < N; n++) {
        st[n] = 1.0 + rnd((st[n] - 1.0) * scale[0]) / scale[0];
        for (int q = 1; q < 4; q++) st[q * N + n] = rnd(st[q * N + n] * scale[1]) / scale[1];
        for (int q = 4; q < 10; q++) st[q * N + n] = rnd(st[q * N + n] * scale[2]) / scale[2];
    }
}

/* nsteps steps in place starting at level t0; storage 0 = exact FP64,
 * 1/2 = round the stored fields after every step (see or_round_storage).   */
int or_run(const or_grid *G, double *st, const double *gf, long t0, int nsteps, int storage,
           const double *scale)
{
    lattice_init();
    const long N = (long)G->nx * G->ny * G->nz;
    double *tmp = (double *)malloc(sizeof(double) * 10 * N);
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; s++) {
        step_r(G, st, tmp, gf, t0 + s);
        if (storage) or_round_storage(G, tmp, storage, scale);
        memcpy(st, tmp, sizeof(double) * 10 * N);
    }
    free(tmp);
    return 0;
}

/* Single-step update at selected fluid nodes only (for sampled checks of
 * large grids): out[q*nidx + k] = new moment q of node idx[k].             */
void or_update_nodes(const or_grid *G, const double *in, const double *gf, const long *idx, long nidx,
                     double *out)
{
    lattice_init();
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nidx; k++) {
        double f[NQ], m[10];
        gather_r(G, in, gf, idx[k], f);
        moments_r(lat(G), f, m);
        for (int q = 0; q < 10; q++) out[q * nidx + k] = m[q];
    }
}

/* FP64 sums over fluid nodes: mass, momentum (3), kinetic energy 1/2 rho u^2.
 * Returns the number of non-finite entries met.                             */
long or_reduce(const or_grid *G, const double *st, double *out)
{
    const long N = (long)G->nx * G->ny * G->nz;
    long bad = 0;
    for (int k = 0; k < 5; k++) out[k] = 0.0;
    for (long n = 0; n < N; n++) {
        if (node_kind(G, n) != NODE_FLUID) continue;
        double rho = st[n], u[3] = {st[N + n], st[2 * N + n], st[3 * N + n]};
        for (int q = 0; q < 10; q++)
            if (!isfinite(st[q * N + n])) bad++;
        out[0] += rho;
        for (int a = 0; a < 3; a++) out[1 + a] += rho * u[a];
        out[4] += 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    }
    return bad;
}

int or_num_threads(void) { return omp_get_max_threads(); }

uint64_t or_splitmix64(uint64_t seed, uint64_t k) { return splitmix64_at(seed, k); }
double or_inlet_xi(uint64_t seed, long t, long n, long N, int a) { return inlet_xi(seed, t, n, N, a); }
double or_inlet_gauss(uint64_t seed, long t, long n, long N, int a) { return inlet_gauss(seed, t, n, N, a); }

/* ------------------------------------------------------------------ */
/* Tangent and adjoint of one step (periodic axes, walls and inflow/outflow
 * ghost layers).  One step maps level t to level t+1: the update of the
 * fluid nodes from every node of level t (ghost nodes being ordinary
 * emitters), then the ghost refill of level t+1 from the new fluid nodes
 * (Section 2.3, Eq. (neq_final)).  Ghost values of level t are inputs of
 * the step like any other node.                                           */

/* Tangent (Jacobian-vector product) of one step by the complex step:
 * dout = d step(st, gf) [dst, dgf].                                        */
int or_jvp_step(const or_grid *G, const double *st, const double *gf, const double *dst, const double *dgf,
                long t, double *dout)
{
    if (G->lattice != 0 && G->lattice != 27) return -3; /* derivatives: D3Q27 only */
    lattice_init();
    const long N = (long)G->nx * G->ny * G->nz;
    double complex *a = (double complex *)malloc(sizeof(double complex) * 10 * N);
    double complex *b = (double complex *)malloc(sizeof(double complex) * 10 * N);
    double complex *g = (double complex *)malloc(sizeof(double complex) * 3 * N);
    if (!a || !b || !g) return -1;
    for (long k = 0; k < 10 * N; k++) a[k] = st[k] + I * CSTEP * dst[k];
    for (long k = 0; k < 3 * N; k++) {
        double g0 = gf ? gf[k] : G->force[k / N];
        double dg = dgf ? dgf[k] : 0.0;
        g[k] = g0 + I * CSTEP * dg;
    }
    step_c(G, a, b, g, t);
    for (long k = 0; k < 10 * N; k++) dout[k] = cimag(b[k]) / CSTEP;
    free(a);
    free(b);
    free(g);
    return 0;
}

/* Adjoint of the moment map at fluid node x: lf[i] = sum_q lam_q dM'_q/df_i,
 * with the populations f arriving at x rebuilt from st.                     */
static void adjoint_populations(const or_grid *G, const double *st, const double *gf, const double *lam,
                                long x, double lf[NQ])
{
    const long N = (long)G->nx * G->ny * G->nz;
    double f[NQ];
    gather_r(G, st, gf, x, f);
    for (int i = 0; i < NQ; i++) {
        double complex fc[NQ], mc[10];
        for (int k = 0; k < NQ; k++) fc[k] = f[k];
        fc[i] += I * CSTEP;
        moments_c(lat(G), fc, mc);
        double s = 0.0;
        for (int q = 0; q < 10; q++) s += lam[q * N + x] * cimag(mc[q]) / CSTEP;
        lf[i] = s;
    }
}

/* Accumulate J^T lf into lm[10] (moments) and lg[3] (force) for the
 * population k emitted by node s: J = d fpost_k / d (M_s, g_s).            */
static void adjoint_emit(const or_grid *G, const double *st, const double *gf, long s, int k, double lf,
                         double lm[10], double lg[3])
{
    const long N = (long)G->nx * G->ny * G->nz;
    double omega = omega_at(G, s);
    for (int p = 0; p < 13; p++) {
        double complex m[10], g[3];
        for (int q = 0; q < 10; q++) m[q] = st[q * N + s];
        for (int a = 0; a < 3; a++) g[a] = gf ? gf[a * N + s] : G->force[a];
        if (p < 10)
            m[p] += I * CSTEP;
        else
            g[p - 10] += I * CSTEP;
        double d = cimag(fpost_c(lat(G), k, m, g, omega, G->order)) / CSTEP;
        if (p < 10)
            lm[p] += d * lf;
        else
            lg[p - 10] += d * lf;
    }
}

/* Transpose of the ghost refill, in place: every ghost node copied its
 * moments from its interior neighbour (all ten, or rho and Pi^neq only on an
 * inlet disc, whose velocity is imposed and does not depend on the state),
 * so its sensitivities are added to that neighbour's and set to zero.
 * Sequential, in node order (several ghosts share a neighbour).             */
static void fold_ghost_sensitivities(const or_grid *G, double *lam)
{
    const long N = (long)G->nx * G->ny * G->nz;
    if (!grid_has_ghosts(G)) return;
    for (long n = 0; n < N; n++) {
        if (node_kind(G, n) != NODE_GHOST) continue;
        int x[3], xf[3];
        double ub[3];
        node_coords(G, n, x);
        interior_neighbour(G, x, xf);
        long nf = node_index(G, xf);
        int imposed = inlet_velocity(G, x, n, 0, ub);
        for (int q = 0; q < 10; q++) {
            if (!(imposed && q >= 1 && q <= 3)) lam[q * N + nf] += lam[q * N + n];
            lam[q * N + n] = 0.0;
        }
    }
}

/* Reverse-mode sensitivity at node y (gather from the downstream nodes):
 * lam_t(y) = sum over populations emitted by y of J^T lam_f, where y emits
 * population i to y + c_i, and, for each direction whose upstream node is
 * solid, its own bounced-back population opp(i) to itself.                 */
static int adjoint_node(const or_grid *G, const double *st, const double *gf, const double *lam1,
                        const double *lf_all, long y, double lm[10], double lg[3])
{
    for (int q = 0; q < 10; q++) lm[q] = 0.0;
    for (int a = 0; a < 3; a++) lg[a] = 0.0;
    const int kind = node_kind(G, y);
    if (kind == NODE_SOLID) return 0; /* walls emit nothing */
    int xy[3];
    node_coords(G, y, xy);
    for (int i = 0; i < NQ; i++) {
        int xd[3], ok = 1;
        for (int d = 0; d < 3; d++) {
            int n = dim(G, d);
            xd[d] = xy[d] + lat(G)->c[i][d];
            if (G->face[2 * d] == FACE_PERIODIC) xd[d] = ((xd[d] % n) + n) % n;
            if (xd[d] < 0 || xd[d] >= n) ok = 0;
        }
        if (ok && node_kind_xyz(G, xd) == NODE_FLUID) {
            long x = node_index(G, xd);
            double lf[NQ];
            if (lf_all)
                memcpy(lf, lf_all + (size_t)x * NQ, sizeof lf);
            else
                adjoint_populations(G, st, gf, lam1, x, lf);
            adjoint_emit(G, st, gf, y, i, lf[i], lm, lg);
        }
        if (kind == NODE_FLUID && upstream(G, xy, i) == -1) { /* bounce-back: y feeds itself */
            double lf[NQ];
            if (lf_all)
                memcpy(lf, lf_all + (size_t)y * NQ, sizeof lf);
            else
                adjoint_populations(G, st, gf, lam1, y, lf);
            adjoint_emit(G, st, gf, y, lat(G)->opp[i], lf[i], lm, lg);
        }
    }
    return 0;
}

/* Full-grid adjoint of one step from level t: lam_t = J_M^T lam_{t+1} and
 * dg += J_g^T lam_{t+1} (dg may be NULL): the ghost refill of level t+1
 * transposed first, then the update.                                       */
int or_adjoint_step(const or_grid *G, const double *st, const double *gf, const double *lam1, double *lam0,
                    double *dg)
{
    if (G->lattice != 0 && G->lattice != 27) return -3; /* derivatives: D3Q27 only */
    lattice_init();
    const long N = (long)G->nx * G->ny * G->nz;
    double *lf_all = (double *)calloc((size_t)N * NQ, sizeof(double));
    double *lamf = (double *)malloc(sizeof(double) * 10 * N);
    if (!lf_all || !lamf) return -1;
    memcpy(lamf, lam1, sizeof(double) * 10 * N);
    fold_ghost_sensitivities(G, lamf);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++)
        if (node_kind(G, x) == NODE_FLUID) adjoint_populations(G, st, gf, lamf, x, lf_all + (size_t)x * NQ);
#pragma omp parallel for schedule(static)
    for (long y = 0; y < N; y++) {
        double lm[10], lg[3];
        adjoint_node(G, st, gf, lamf, lf_all, y, lm, lg);
        for (int q = 0; q < 10; q++) lam0[q * N + y] = lm[q];
        if (dg)
            for (int a = 0; a < 3; a++) dg[a * N + y] += lg[a];
    }
    free(lf_all);
    free(lamf);
    return 0;
}

/* Adjoint of one step at selected nodes only: lam_out[q*nidx+k], dg_out[a*nidx+k]. */
int or_adjoint_nodes(const or_grid *G, const double *st, const double *gf, const double *lam1, const long *idx,
                     long nidx, double *lam_out, double *dg_out)
{
    if (G->lattice != 0 && G->lattice != 27) return -3; /* derivatives: D3Q27 only */
    lattice_init();
    const long N = (long)G->nx * G->ny * G->nz;
    double *lamf = NULL;
    if (grid_has_ghosts(G)) {
        lamf = (double *)malloc(sizeof(double) * 10 * N);
        if (!lamf) return -1;
        memcpy(lamf, lam1, sizeof(double) * 10 * N);
        fold_ghost_sensitivities(G, lamf);
    }
    const double *lam = lamf ? lamf : lam1;
#pragma omp parallel for schedule(dynamic, 4)
    for (long k = 0; k < nidx; k++) {
        double lm[10], lg[3];
        adjoint_node(G, st, gf, lam, NULL, idx[k], lm, lg);
        for (int q = 0; q < 10; q++) lam_out[q * nidx + k] = lm[q];
        for (int a = 0; a < 3; a++) dg_out[a * nidx + k] = lg[a];
    }
    free(lamf);
    return 0;
}

/* Kinetic-energy objective L = 1/2 sum_fluid rho |u|^2 and its gradient
 * with respect to the stored moments (rho, u, Pi).                          */
double or_ke_seed(const or_grid *G, const double *st, double *lam)
{
    const long N = (long)G->nx * G->ny * G->nz;
    double L = 0.0;
    memset(lam, 0, sizeof(double) * 10 * N);
    for (long n = 0; n < N; n++) {
        if (node_kind(G, n) != NODE_FLUID) continue;
        double rho = st[n], u2 = 0.0;
        for (int a = 0; a < 3; a++) u2 += st[(1 + a) * N + n] * st[(1 + a) * N + n];
        L += 0.5 * rho * u2;
        lam[n] = 0.5 * u2;
        for (int a = 0; a < 3; a++) lam[(1 + a) * N + n] = rho * st[(1 + a) * N + n];
    }
    return L;
}

/* Wall shear objective: the x-directed viscous force on the walls normal to
 * y and z, L = sum over fluid nodes next to such a wall face f of
 * s_f sigma_xd, with d the face's normal axis, s_f = +1 on the low face and
 * -1 on the high face, and the viscous stress of the BGK update
 * sigma = -(1 - omega / 2) Pi^neq (Pi^neq the stored pre-collision
 * non-equilibrium moment, omega that of the node).  L is linear in Pi, so
 * lam = dL/dM is the constant -s_f (1 - omega / 2) on Pi_xd of those nodes
 * (summed over the faces a node touches).  Returns L.                       */
double or_wall_shear_seed(const or_grid *G, const double *st, double *lam)
{
    const long N = (long)G->nx * G->ny * G->nz;
    double L = 0.0;
    memset(lam, 0, sizeof(double) * 10 * N);
    for (long n = 0; n < N; n++) {
        if (node_kind(G, n) != NODE_FLUID) continue;
        int x[3];
        node_coords(G, n, x);
        const double k = 1.0 - 0.5 * omega_at(G, n);
        for (int f = 2; f < 6; f++) {
            if (G->face[f] != FACE_WALL) continue;
            const int d = f / 2;
            const int layer = (f % 2 == 0) ? 1 : dim(G, d) - 2;
            if (x[d] != layer) continue;
            const double s = (f % 2 == 0) ? 1.0 : -1.0;
            const int q = 4 + PI_IDX[0][d]; /* Pi_xy or Pi_xz */
            L += -s * k * st[q * N + n];
            lam[q * N + n] += -s * k;
        }
    }
    return L;
}

/* Gradient of L(state after nsteps) with respect to the initial state and the
 * force field, by storing every level and sweeping the adjoint backwards.
 * objective 0: kinetic energy (or_ke_seed); 1: wall shear (or_wall_shear_seed).
 * lam0 (10N) receives dL/dM_0; dg (3N, may be NULL) receives dL/dg.  The
 * ghost layers of the initial state are refilled from its interior (level
 * t0) first, so L is a function of the interior and of the force field, and
 * lam0 is zero on ghost nodes.                                              */
int or_rollout_grad(const or_grid *G, const double *st0, const double *gf, long t0, int nsteps, int objective,
                    double *loss, double *lam0, double *dg)
{
    if (G->lattice != 0 && G->lattice != 27) return -3; /* derivatives: D3Q27 only */
    lattice_init();
    const long N = (long)G->nx * G->ny * G->nz;
    double *traj = (double *)malloc(sizeof(double) * 10 * N * (size_t)(nsteps + 1));
    double *lam = (double *)malloc(sizeof(double) * 10 * N);
    double *tmp = (double *)malloc(sizeof(double) * 10 * N);
    if (!traj || !lam || !tmp) return -1;
    memcpy(traj, st0, sizeof(double) * 10 * N);
    ghost_fill_r(G, traj, t0);
    for (int s = 0; s < nsteps; s++)
        step_r(G, traj + (size_t)s * 10 * N, traj + (size_t)(s + 1) * 10 * N, gf, t0 + s);
    *loss = objective == 1 ? or_wall_shear_seed(G, traj + (size_t)nsteps * 10 * N, lam)
                           : or_ke_seed(G, traj + (size_t)nsteps * 10 * N, lam);
    if (dg) memset(dg, 0, sizeof(double) * 3 * N);
    for (int s = nsteps - 1; s >= 0; s--) {
        or_adjoint_step(G, traj + (size_t)s * 10 * N, gf, lam, tmp, dg);
        memcpy(lam, tmp, sizeof(double) * 10 * N);
    }
    fold_ghost_sensitivities(G, lam); /* the refill of the initial level */
    memcpy(lam0, lam, sizeof(double) * 10 * N);
    free(traj);
    free(lam);
    free(tmp);
    return 0;
}
