/* Runs the FP64 oracle (test infrastructure) over every boundary rule on
 * small and ragged grids, for a host build with AddressSanitizer and
 * UndefinedBehaviorSanitizer; prints "ok" when every run stays finite. */
#include "../../oracle/mrt_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static void side(orc_side *s, int lo, int hi, double split0, double rate, const double st_lo[4],
                 const double st_hi[4])
{
    s->kind_lo = lo;
    s->kind_hi = hi;
    for (int c = 0; c < 4; ++c) {
        s->state_lo[c] = st_lo[c];
        s->state_hi[c] = st_hi[c];
    }
    s->split0 = split0;
    s->split_rate = rate;
}

static int run_case(const orc_model *m, int nx, int ny, int set)
{
    const double a[4] = {1.0, 0.1, 0.0, 1.0}, b[4] = {0.5, 0.0, 0.1, 0.8}, w[4] = {1.0, 0.05, 0.0, 1.0};
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.dx = p.dy = 2e-3;
    p.dt = 1e-5;
    for (int k = 4; k < NQ; ++k) p.s[k] = 1e4 + 500.0 * k;
    const double inf = 1e300;
    switch (set) {
    case 0:  /* periodic everywhere */
        for (int k = 0; k < 4; ++k) side(&p.side[k], ORC_PERIODIC, ORC_PERIODIC, inf, 0, a, a);
        break;
    case 1:  /* prescribed x ends, periodic y */
        side(&p.side[0], ORC_DIRICHLET, ORC_DIRICHLET, inf, 0, a, a);
        side(&p.side[1], ORC_DIRICHLET, ORC_DIRICHLET, inf, 0, b, b);
        side(&p.side[2], ORC_PERIODIC, ORC_PERIODIC, inf, 0, a, a);
        side(&p.side[3], ORC_PERIODIC, ORC_PERIODIC, inf, 0, a, a);
        break;
    case 2:  /* extrapolation and reflection */
        side(&p.side[0], ORC_EXTRAPOLATE, ORC_EXTRAPOLATE, inf, 0, a, a);
        side(&p.side[1], ORC_EXTRAPOLATE, ORC_EXTRAPOLATE, inf, 0, a, a);
        side(&p.side[2], ORC_REFLECT, ORC_REFLECT, inf, 0, a, a);
        side(&p.side[3], ORC_REFLECT, ORC_REFLECT, inf, 0, a, a);
        break;
    default: /* walls and a switch point that moves */
        side(&p.side[0], ORC_PERIODIC, ORC_PERIODIC, inf, 0, a, a);
        side(&p.side[1], ORC_PERIODIC, ORC_PERIODIC, inf, 0, a, a);
        side(&p.side[2], ORC_WALL, ORC_WALL, inf, 0, w, w);
        side(&p.side[3], ORC_DIRICHLET, ORC_EXTRAPOLATE, 0.4 * nx * p.dx, 5.0, b, a);
        break;
    }
    const size_t cells = (size_t)nx * ny, n = (size_t)(nx + 2) * (ny + 2) * NQ;
    double *rho = malloc(cells * sizeof(double)), *ux = malloc(cells * sizeof(double));
    double *uy = malloc(cells * sizeof(double)), *T = malloc(cells * sizeof(double));
    double *pr = malloc(cells * sizeof(double));
    double *f = calloc(n, sizeof(double)), *work = calloc(n, sizeof(double));
    for (size_t c = 0; c < cells; ++c) {
        rho[c] = 1.0 + 0.1 * (double)(c % 7) / 7.0;
        ux[c] = 0.05 * (double)(c % 5) / 5.0;
        uy[c] = -0.03 * (double)(c % 3) / 3.0;
        T[c] = 1.0 + 0.05 * (double)(c % 11) / 11.0;
    }
    orc_init_macro(m, &p, rho, ux, uy, T, f);
    double out[16] = {0}, sums[4];
    orc_run(m, &p, f, work, 0, 25, 1, out);
    orc_sums(m, &p, f, sums);
    orc_read_macro(m, &p, f, rho, ux, uy, T, pr);
    int bad = 0;
    for (int k = 0; k < 4; ++k) bad |= !isfinite(sums[k]);
    for (int k = 0; k < 16; ++k) bad |= !isfinite(out[k]);
    for (size_t c = 0; c < cells; ++c) bad |= !isfinite(rho[c]) || !isfinite(pr[c]);
    free(rho); free(ux); free(uy); free(T); free(pr); free(f); free(work);
    if (bad) fprintf(stderr, "non-finite result: %dx%d, set %d\n", nx, ny, set);
    return bad;
}

int main(void)
{
    orc_model m;
    if (orc_model_init(&m) != 0) return 2;
    const int shapes[][2] = {{3, 3}, {4, 3}, {3, 5}, {17, 5}, {33, 9}};
    int bad = 0;
    for (unsigned s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
        for (int set = 0; set < 4; ++set) bad |= run_case(&m, shapes[s][0], shapes[s][1], set);
    double fh[NQ], C[NQ], feq[NQ], q[5];
    double sr[NQ];
    for (int k = 0; k < NQ; ++k) sr[k] = 1e3 * k;
    orc_feq_velocity(&m, 1.3, 0.2, -0.1, 0.9, feq);
    orc_moments(&m, feq, fh);
    orc_collision(&m, sr, feq, C);
    orc_macro_of(&m, feq, q);
    for (int k = 0; k < NQ; ++k) bad |= !isfinite(C[k]) || !isfinite(fh[k]);
    if (bad) return 1;
    printf("ok\n");
    return 0;
}
