/* Host-only AddressSanitizer / UndefinedBehaviorSanitizer run of the FP64
   oracle (test infrastructure): every exported entry point on small grids
   with each boundary kind, lattice, Hermite order and option.  Built and run
   by test_oracle_sanitizers.py; the oracle source is compiled in directly. */
#include "../oracle/tslb_oracle.c"
#include <stdio.h>
#include <stdlib.h>

static double frand(unsigned *s) { *s = *s * 1664525u + 1013904223u; return ((*s >> 8) & 0xffffff) / 16777216.0 - 0.5; }

static void fill(double *st, long N, unsigned seed, int d2)
{
    for (long n = 0; n < N; n++) {
        st[n] = 1.0 + 0.01 * frand(&seed);
        for (int k = 1; k < 10; k++) st[k * N + n] = (k < 4 ? 0.03 : 1e-3) * frand(&seed);
        if (d2) { st[3 * N + n] = 0; st[6 * N + n] = 0; st[8 * N + n] = 0; st[9 * N + n] = 0; }
    }
}

static int run_case(int nx, int ny, int nz, const int face[6], int lattice, int order, int noise_kind, int sponge)
{
    or_grid G = {0};
    G.nx = nx; G.ny = ny; G.nz = nz;
    for (int f = 0; f < 6; f++) G.face[f] = face[f];
    G.tau = 0.6; G.force[0] = 1e-6; G.order = order; G.noise_kind = noise_kind; G.lattice = lattice;
    G.inlet_u[0] = 0.05; G.inlet_center[0] = ny / 2.0; G.inlet_center[1] = nz / 2.0; G.inlet_radius = 2.5;
    G.inlet_noise = 0.02; G.seed = 42;
    double *tz = NULL;
    if (sponge) { tz = malloc(sizeof(double) * nz); for (int z = 0; z < nz; z++) tz[z] = 0.6 + 0.01 * z; G.tau_z = tz; }
    const long N = (long)nx * ny * nz;
    double *a = malloc(sizeof(double) * 10 * N), *b = malloc(sizeof(double) * 10 * N);
    double *gf = malloc(sizeof(double) * 3 * N), *l1 = malloc(sizeof(double) * 10 * N), *l0 = malloc(sizeof(double) * 10 * N);
    double *dg = calloc(3 * N, sizeof(double)), *dout = malloc(sizeof(double) * 10 * N), *upd = malloc(sizeof(double) * 10 * 7);
    unsigned s = 7;
    fill(a, N, 3, lattice == 9);
    for (long i = 0; i < 3 * N; i++) gf[i] = (lattice == 9 && i >= 2 * N) ? 0.0 : 1e-6 * frand(&s);
    or_ghost_fill(&G, a, 0);
    or_step(&G, a, b, gf, 0);
    or_step(&G, a, b, NULL, 0);
    long idx[7] = {0, 1, N / 3, N / 2, N - 2, N - 1, N / 5};
    or_update_nodes(&G, a, gf, idx, 7, upd);
    double red[5];
    or_reduce(&G, b, red);
    double sc[3] = {1, 1, 1};
    for (int k = 0; k < 3; k++) { double *c = malloc(sizeof(double) * 10 * N); for (long i = 0; i < 10 * N; i++) c[i] = a[i]; or_run(&G, c, NULL, 0, 3, k, sc); free(c); }
    signed char *kinds = malloc(N);
    or_node_kinds(&G, kinds);
    int rc = 0;
    if (lattice == 27 && order == 3) {
        fill(l1, N, 5, 0);
        or_adjoint_step(&G, a, gf, l1, l0, dg);
        or_jvp_step(&G, a, gf, l1, NULL, 0, dout);
        { double dgn[21]; or_adjoint_nodes(&G, a, gf, l1, idx, 7, upd, dgn); }
        double loss;
        int ghosts = 0;
        for (int f = 0; f < 6; f++) ghosts |= is_ghost_face(face[f]);
        if (!ghosts) {
            rc |= or_rollout_grad(&G, a, gf, 0, 4, 0, &loss, l0, dg);
            rc |= or_rollout_grad(&G, a, gf, 0, 4, 1, &loss, l0, dg);
            or_ke_seed(&G, a, l0);
            or_wall_shear_seed(&G, a, l0);
        }
    }
    free(a); free(b); free(gf); free(l1); free(l0); free(dg); free(dout); free(upd); free(kinds); free(tz);
    return rc;
}

int main(void)
{
    const int P[6] = {0, 0, 0, 0, 0, 0}, W[6] = {0, 0, 1, 1, 0, 0}, WA[6] = {1, 1, 1, 1, 1, 1}, J[6] = {2, 3, 3, 3, 3, 3},
              PJ[6] = {0, 0, 0, 0, 2, 3};
    int rc = 0;
    for (int order = 2; order <= 3; order++) {
        rc |= run_case(7, 6, 5, P, 27, order, 0, 0);
        rc |= run_case(7, 6, 5, W, 27, order, 0, 0);
        rc |= run_case(5, 6, 7, WA, 27, order, 0, 0);
        rc |= run_case(7, 6, 5, J, 27, order, 0, 0);
        rc |= run_case(6, 5, 8, PJ, 27, order, 1, 1);
        rc |= run_case(7, 6, 5, W, 19, order, 0, 0);
        rc |= run_case(7, 6, 5, J, 19, order, 1, 0);
        rc |= run_case(9, 7, 1, P, 9, order, 0, 0);
        const int W2[6] = {1, 1, 1, 1, 0, 0}, J2[6] = {2, 3, 0, 0, 0, 0};
        rc |= run_case(9, 7, 1, W2, 9, order, 0, 0);
        rc |= run_case(9, 7, 1, J2, 9, order, 1, 0);
    }
    printf("sanitizer run done, rc %d\n", rc);
    return rc != 0;
}
