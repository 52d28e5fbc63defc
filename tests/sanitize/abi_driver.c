/* Calls every entry point of include/mrtfd.h that needs no GPU -- parameter
 * validation (valid and invalid sets, message buffers of every length),
 * workspace sizes, the model, status strings and NULL arguments -- for a
 * host build of the library with AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Prints "ok" when every result is as the
 * header states. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "../../include/mrtfd.h"

static int fails = 0;
#define EXPECT(c)                                                                 \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #c);      \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

static mrtfd_params valid(void)
{
    mrtfd_params p;
    memset(&p, 0, sizeof p);
    p.nx = 130;
    p.ny = 70;
    p.dx = p.dy = 2e-3;
    p.dt = 1e-5;
    for (int k = 4; k < 16; ++k) p.s[k] = 1e4;
    for (int k = 0; k < 4; ++k) {
        p.side[k].kind_lo = p.side[k].kind_hi = MRTFD_BC_PERIODIC;
        p.side[k].split0 = 1e300;
        for (int c = 0; c < 4; ++c) p.side[k].state_lo[c] = p.side[k].state_hi[c] = c == 0 || c == 3;
    }
    p.graph_steps = 64;
    return p;
}

static int check(const mrtfd_params *p)
{
    char msg[256];
    const int32_t r = mrtfd_check_params(p, msg, sizeof msg);
    /* every message length, including none */
    for (size_t len = 0; len < 40; ++len) {
        char small[40];
        memset(small, 'x', sizeof small);
        EXPECT(mrtfd_check_params(p, len ? small : NULL, len) == r);
        if (len) EXPECT(memchr(small, 0, len) != NULL);
    }
    return r;
}

int main(void)
{
    size_t ps = 0, ss = 0;
    EXPECT(mrtfd_struct_sizes(&ps, &ss) == MRTFD_OK);
    EXPECT(ps == sizeof(mrtfd_params) && ss == sizeof(mrtfd_side));

    double v[32], M[256], Mi[256];
    EXPECT(mrtfd_model(v, M, Mi) == MRTFD_OK);
    double worst = 0.0;
    for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) {
            double s = 0.0;
            for (int k = 0; k < 16; ++k) s += M[i * 16 + k] * Mi[k * 16 + j];
            worst = fmax(worst, fabs(s - (i == j)));
        }
    EXPECT(worst < 1e-12);

    mrtfd_params p = valid();
    EXPECT(check(&p) == MRTFD_OK);
    EXPECT(mrtfd_workspace_bytes(&p) > 0);
    EXPECT(check(NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_workspace_bytes(NULL) == 0);

    /* one bad field at a time */
    p = valid(); p.nx = 2;                         EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.ny = -5;                        EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.dx = 0.0;                       EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.dt = NAN;                       EXPECT(check(&p) != MRTFD_OK);
    p = valid(); p.s[7] = -1.0;                    EXPECT(check(&p) != MRTFD_OK);
    p = valid(); p.s[9] = 2e5;                     EXPECT(check(&p) == MRTFD_ERR_UNSTABLE);
    p = valid(); p.dt = 1e-3;                      EXPECT(check(&p) == MRTFD_ERR_UNSTABLE);
    p = valid(); p.side[0].kind_lo = 9;            EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.side[1].kind_lo = p.side[1].kind_hi = MRTFD_BC_REFLECT;
    EXPECT(check(&p) == MRTFD_ERR_ARG);            /* periodic west needs periodic east */
    p = valid(); p.precision = 7;                  EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.kernel = 11;                    EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.rows = 5;                       EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.layout = 3;                     EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.graph_steps = -1;               EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.flux_budget = 2;                EXPECT(check(&p) == MRTFD_ERR_ARG);
    p = valid(); p.collision = MRTFD_COLLISION_SRT; EXPECT(check(&p) == MRTFD_OK);
    p.s[6] = 2e4;                                  EXPECT(check(&p) == MRTFD_ERR_ARG);  /* SRT needs equal rates */
    p = valid(); p.nx = 100000; p.ny = 100000;     EXPECT(check(&p) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_workspace_bytes(&p) == 0);

    /* NULL contexts and arguments */
    p = valid();
    mrtfd_ctx *ctx = (mrtfd_ctx *)0;
    EXPECT(mrtfd_create(&p, NULL, 0, NULL, &ctx) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_create(NULL, NULL, 0, NULL, &ctx) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_destroy(NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_step(NULL, 1) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_init_macro(NULL, NULL, NULL, NULL, NULL) == MRTFD_ERR_ARG);
    double sums[4];
    EXPECT(mrtfd_sums(NULL, sums) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_last_error(NULL) != NULL);
    for (int32_t code = -8; code <= 1; ++code) {
        const char *s = mrtfd_status_string(code);
        EXPECT(s != NULL && strlen(s) > 0);
    }

    /* batches */
    mrtfd_batch_params bp;
    memset(&bp, 0, sizeof bp);
    bp.ntubes = 3;
    bp.dx = 2e-3;
    bp.dt = 1e-5;
    for (int k = 4; k < 16; ++k) bp.s[k] = 1e4;
    const int32_t n[3] = {200, 331, 64};
    EXPECT(mrtfd_batch_workspace_bytes(&bp, n) > 0);
    const int32_t nbad[3] = {200, 2, 64};
    EXPECT(mrtfd_batch_workspace_bytes(&bp, nbad) == 0);
    EXPECT(mrtfd_batch_workspace_bytes(NULL, n) == 0);
    bp.seg_cols = 50;
    EXPECT(mrtfd_batch_workspace_bytes(&bp, n) == 0);
    mrtfd_batch *b = (mrtfd_batch *)0;
    EXPECT(mrtfd_batch_create(NULL, n, NULL, NULL, NULL, NULL, 0, NULL, &b) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_batch_destroy(NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_batch_last_error(NULL) != NULL);

    /* the von Neumann screen: validation before any HIP call */
    p = valid();
    const double st[4] = {1.0, 0.0, 0.0, 1.0}, bad[4] = {1.0, 0.0, 0.0, -1.0};
    double *d = (double *)(uintptr_t)8; /* never dereferenced: every case returns before a launch */
    EXPECT(mrtfd_screen(&p, st, d, 0, d, d, NULL) == MRTFD_OK);
    EXPECT(mrtfd_screen(&p, st, d, -1, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen(&p, st, NULL, 4, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen(&p, st, d, 4, NULL, NULL, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen(&p, bad, d, 4, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen(NULL, st, d, 4, d, d, NULL) == MRTFD_ERR_ARG);
    p.dt = 1e-3;  /* dt s beyond 1: refused by create, accepted by the screen */
    EXPECT(mrtfd_screen(&p, st, d, 0, d, d, NULL) == MRTFD_OK);
    p.dy = 0.0;
    EXPECT(mrtfd_screen(&p, st, d, 4, d, d, NULL) == MRTFD_ERR_ARG);
    p = valid();
    EXPECT(mrtfd_screen_sets(&p, 0, d, d, d, 4, d, d, NULL) == MRTFD_OK);
    EXPECT(mrtfd_screen_sets(&p, -1, d, d, d, 4, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen_sets(&p, 1 << 16, d, d, d, 1 << 15, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen_sets(&p, 3, NULL, d, d, 4, d, d, NULL) == MRTFD_ERR_ARG);
    EXPECT(mrtfd_screen_sets(&p, 3, d, d, d, 4, NULL, NULL, NULL) == MRTFD_ERR_ARG);

    if (fails) return 1;
    printf("ok\n");
    return 0;
}
