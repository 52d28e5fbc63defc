/*
 * Plain FP64 CPU oracle for the energy-conserving multiple-relaxation-time
 * finite-difference lattice Boltzmann (MRT-FDLB) step of Chen, Xu, Zhang and
 * Li, "Multiple-relaxation-time lattice Boltzmann model for compressible
 * fluids" (arXiv:0908.3749).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the product path
 * never does.  It shares no code, header, table or constant with the GPU
 * library: the velocity set, the matrix M, its inverse, the equilibria, the
 * collision, the stencil and the boundary rules are written here again from
 * the paper.
 *
 * Everything is double precision, written in the paper's order and notation,
 * with no blocking, fusion or reordering beyond what the paper states.
 * Indices in comments are the paper's (1-based); arrays are 0-based.
 *
 * Layout: a grid of nx*ny interior cells plus one ghost cell on each side,
 * stored cell-major, f[((j+1)*(nx+2) + (i+1))*16 + q] for interior i in
 * [0,nx), j in [0,ny) and population q in [0,16).  Corner ghosts are never
 * read (the difference stencil has no cross term).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 16

/* Boundary rule kinds (the paper's "macroscopic variable boundary
 * conditions", Sect. V).  Values are this oracle's own. */
enum {
    ORC_PERIODIC = 0,    /* wrap to the opposite interior edge (Sect. V.A) */
    ORC_DIRICHLET = 1,   /* f = f^eq of a prescribed (rho,u1,u2,T)         */
    ORC_REFLECT = 2,     /* interior state with normal velocity reversed   */
    ORC_EXTRAPOLATE = 3, /* linear extrapolation of (rho,u1,u2,T)          */
    ORC_WALL = 4         /* wall speed and temperature, density of fluid   */
};

typedef struct {
    int32_t kind_lo, kind_hi; /* rule where along-side coordinate <= split, > split */
    double state_lo[4];       /* rho, u1, u2, T */
    double state_hi[4];
    double split0, split_rate; /* split(t) = split0 + split_rate * t */
} orc_side;

typedef struct {
    int32_t nx, ny;
    double dx, dy, dt;
    double s[NQ];      /* diagonal of S-hat, s_1..s_16 */
    orc_side side[4];  /* 0 west (i=-1), 1 east (i=nx), 2 south (j=-1), 3 north (j=ny) */
} orc_params;

typedef struct {
    double v[NQ][2];     /* discrete velocities, Eq. (4) */
    double M[NQ][NQ];    /* M[k][i] = m_{k+1}(v_i), Eq. (5a)-(5p) */
    double Minv[NQ][NQ]; /* inverse of M */
} orc_model;

/* ------------------------------------------------------------------------
 * Velocity set, Eq. (4).  Four groups of four: cyc(+-1,0), cyc(+-6,0),
 * sqrt2(+-1,+-1), (3/sqrt2)(+-1,+-1).  The order inside each group is the one
 * the printed rows m_2 and m_3 of M fix (Sect. III.A): the axis groups run
 * (+,0),(0,+),(-,0),(0,-) and the diagonal groups (+,+),(-,+),(-,-),(+,-).
 * ---------------------------------------------------------------------- */
void orc_velocities(double v[NQ][2])
{
    static const double ax[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    static const double dg[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    const double r2 = sqrt(2.0), r3 = 3.0 / sqrt(2.0);
    for (int k = 0; k < 4; ++k) {
        v[k][0] = ax[k][0];
        v[k][1] = ax[k][1];
        v[4 + k][0] = 6.0 * ax[k][0];
        v[4 + k][1] = 6.0 * ax[k][1];
        v[8 + k][0] = r2 * dg[k][0];
        v[8 + k][1] = r2 * dg[k][1];
        v[12 + k][0] = r3 * dg[k][0];
        v[12 + k][1] = r3 * dg[k][1];
    }
}

/* ------------------------------------------------------------------------
 * Transformation matrix M, Eq. (5a)-(5p): row k is the polynomial m_k
 * evaluated at every discrete velocity.
 * ---------------------------------------------------------------------- */
void orc_build_M(const double v[NQ][2], double M[NQ][NQ])
{
    for (int i = 0; i < NQ; ++i) {
        const double x = v[i][0], y = v[i][1];
        const double x2 = x * x, y2 = y * y, q = x2 + y2;
        M[0][i] = 1.0;                               /* (5a) */
        M[1][i] = x;                                 /* (5b) */
        M[2][i] = y;                                 /* (5c) */
        M[3][i] = q / 2.0;                           /* (5d) */
        M[4][i] = x2 - y2;                           /* (5e) */
        M[5][i] = x * y;                             /* (5f) */
        M[6][i] = x * q / 2.0;                       /* (5g) */
        M[7][i] = y * q / 2.0;                       /* (5h) */
        M[8][i] = x * (x2 - 3.0 * y2);               /* (5i) */
        M[9][i] = y * (3.0 * x2 - y2);               /* (5j) */
        M[10][i] = q * q / 4.0;                      /* (5k) */
        M[11][i] = x2 * x2 - 6.0 * x2 * y2 + y2 * y2; /* (5l) */
        M[12][i] = q * (x2 - y2);                    /* (5m) */
        M[13][i] = q * x * y;                        /* (5n) */
        M[14][i] = x * (x2 - 3.0 * y2) * q;          /* (5o) */
        M[15][i] = y * (3.0 * x2 - y2) * q;          /* (5p) */
    }
}

/* ------------------------------------------------------------------------
 * Matrix inverse by Gauss-Jordan elimination with partial pivoting.  The
 * paper uses f = M^-1 f-hat (Sect. II) without printing M^-1.
 * Returns 0 on success, -1 if a pivot vanishes.
 * ---------------------------------------------------------------------- */
int orc_invert(int n, const double *A, double *Ainv)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(2 * n));
    if (!a) return -1;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * 2 * n + c]) > fabs(a[piv * 2 * n + c])) piv = r;
        if (a[piv * 2 * n + c] == 0.0) {
            free(a);
            return -1;
        }
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) {
                double t = a[c * 2 * n + k];
                a[c * 2 * n + k] = a[piv * 2 * n + k];
                a[piv * 2 * n + k] = t;
            }
        const double p = a[c * 2 * n + c];
        for (int k = 0; k < 2 * n; ++k) a[c * 2 * n + k] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double m = a[r * 2 * n + c];
            if (m == 0.0) continue;
            for (int k = 0; k < 2 * n; ++k) a[r * 2 * n + k] -= m * a[c * 2 * n + k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = a[r * 2 * n + n + c];
    free(a);
    return 0;
}

int orc_model_init(orc_model *m)
{
    orc_velocities(m->v);
    orc_build_M(m->v, m->M);
    return orc_invert(NQ, &m->M[0][0], &m->Minv[0][0]);
}

/* ------------------------------------------------------------------------
 * Equilibria of the moments.  The conserved moments are rho, j_x, j_y, e
 * (Sect. III.A); the nonconserved ones follow Eq. (14a)-(14i), with
 * f-hat_12^eq = f-hat_15^eq = f-hat_16^eq = 0.  The pressure is
 * P = e - (j_x^2 + j_y^2) / (2 rho) (the model's ideal-gas equation of state
 * with R = 1: e = rho (T + |u|^2 / 2) and P = rho T).
 * ---------------------------------------------------------------------- */
void orc_feq_moments(double rho, double jx, double jy, double e, double out[NQ])
{
    const double P = e - (jx * jx + jy * jy) / (2.0 * rho);
    const double jx2 = jx * jx, jy2 = jy * jy, j2 = jx2 + jy2;
    out[0] = rho;
    out[1] = jx;
    out[2] = jy;
    out[3] = e;
    out[4] = (jx2 - jy2) / rho;                                     /* (14a) */
    out[5] = jx * jy / rho;                                         /* (14b) */
    out[6] = (e + P) * jx / rho;                                    /* (14c) */
    out[7] = (e + P) * jy / rho;                                    /* (14d) */
    out[8] = (jx2 - 3.0 * jy2) * jx / (rho * rho);                  /* (14e) */
    out[9] = (3.0 * jx2 - jy2) * jy / (rho * rho);                  /* (14f) */
    out[10] = 2.0 * e * e / rho - j2 * j2 / (4.0 * rho * rho * rho); /* (14g) */
    out[11] = 0.0;
    out[12] = (6.0 * rho * e - 2.0 * jx2 - 2.0 * jy2) * (jx2 - jy2) / (rho * rho * rho); /* (14h) */
    out[13] = (6.0 * rho * e - 2.0 * jx2 - 2.0 * jy2) * jx * jy / (rho * rho * rho);     /* (14i) */
    out[14] = 0.0;
    out[15] = 0.0;
}

/* f-hat = M f (Sect. II). */
void orc_moments(const orc_model *m, const double f[NQ], double fh[NQ])
{
    for (int k = 0; k < NQ; ++k) {
        double acc = 0.0;
        for (int i = 0; i < NQ; ++i) acc += m->M[k][i] * f[i];
        fh[k] = acc;
    }
}

/* Velocity-space equilibrium f^eq = M^-1 f-hat^eq of a macroscopic state
 * (rho, u1, u2, T), with j = rho u and e = rho (T + |u|^2 / 2). */
void orc_feq_velocity(const orc_model *m, double rho, double ux, double uy, double T,
                      double out[NQ])
{
    double fh[NQ];
    const double e = rho * (T + 0.5 * (ux * ux + uy * uy));
    orc_feq_moments(rho, rho * ux, rho * uy, e, fh);
    for (int i = 0; i < NQ; ++i) {
        double acc = 0.0;
        for (int k = 0; k < NQ; ++k) acc += m->Minv[i][k] * fh[k];
        out[i] = acc;
    }
}

/* Macroscopic state of one node: rho, u1, u2, T and p = rho T from the
 * conserved moments f-hat_1..4. */
void orc_macro_of(const orc_model *m, const double f[NQ], double q[5])
{
    double fh[NQ];
    orc_moments(m, f, fh);
    const double rho = fh[0], jx = fh[1], jy = fh[2], e = fh[3];
    const double P = e - (jx * jx + jy * jy) / (2.0 * rho);
    q[0] = rho;
    q[1] = jx / rho;
    q[2] = jy / rho;
    q[3] = P / rho;
    q[4] = P;
}

/* ------------------------------------------------------------------------
 * Collision term of Eq. (3): C_i = sum_l M^-1_il s_l (f-hat_l - f-hat_l^eq).
 * For the conserved moments f-hat^eq equals f-hat, so their difference is
 * exactly zero whatever s_1..s_4 hold.
 * ---------------------------------------------------------------------- */
void orc_collision(const orc_model *m, const double s[NQ], const double f[NQ], double C[NQ])
{
    double fh[NQ], feq[NQ], d[NQ];
    orc_moments(m, f, fh);
    orc_feq_moments(fh[0], fh[1], fh[2], fh[3], feq);
    for (int l = 0; l < NQ; ++l) d[l] = s[l] * (fh[l] - feq[l]);
    for (int i = 0; i < NQ; ++i) {
        double acc = 0.0;
        for (int l = 0; l < NQ; ++l) acc += m->Minv[i][l] * d[l];
        C[i] = acc;
    }
}

/* ------------------------------------------------------------------------
 * One cell update: forward Euler in time, Eq. (A.1a), with the Lax-Wendroff
 * space difference of Eq. (A.1b), and the collision evaluated at the same
 * time level (the unsplit update of the stability analysis, Sect. IV):
 *   f_i(t+dt) = f_i - dt [v_i . grad f_i]_A.1b - dt C_i(f).
 * fE/fW/fN/fS are the neighbours at x+dx, x-dx, y+dy, y-dy.
 * ---------------------------------------------------------------------- */
void orc_cell_update(const orc_model *m, const orc_params *p, const double fc[NQ],
                     const double fE[NQ], const double fW[NQ], const double fN[NQ],
                     const double fS[NQ], double out[NQ])
{
    double C[NQ];
    const double dx = p->dx, dy = p->dy, dt = p->dt;
    orc_collision(m, p->s, fc, C);
    for (int i = 0; i < NQ; ++i) {
        const double vx = m->v[i][0], vy = m->v[i][1];
        const double grad = vx * (fE[i] - fW[i]) / (2.0 * dx)
                          + vy * (fN[i] - fS[i]) / (2.0 * dy)
                          - vx * vx * dt * (fE[i] - 2.0 * fc[i] + fW[i]) / (2.0 * dx * dx)
                          - vy * vy * dt * (fN[i] - 2.0 * fc[i] + fS[i]) / (2.0 * dy * dy);
        out[i] = fc[i] - dt * grad - dt * C[i];
    }
}

/* ------------------------------------------------------------------------
 * Grid helpers.
 * ---------------------------------------------------------------------- */
static inline size_t cell(const orc_params *p, int i, int j)
{
    return ((size_t)(j + 1) * (size_t)(p->nx + 2) + (size_t)(i + 1)) * NQ;
}

void orc_init_macro(const orc_model *m, const orc_params *p, const double *rho,
                    const double *ux, const double *uy, const double *T, double *f)
{
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            const size_t c = (size_t)j * p->nx + i;
            orc_feq_velocity(m, rho[c], ux[c], uy[c], T[c], f + cell(p, i, j));
        }
}

void orc_read_macro(const orc_model *m, const orc_params *p, const double *f, double *rho,
                    double *ux, double *uy, double *T, double *pr)
{
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double q[5];
            const size_t c = (size_t)j * p->nx + i;
            orc_macro_of(m, f + cell(p, i, j), q);
            rho[c] = q[0];
            ux[c] = q[1];
            uy[c] = q[2];
            T[c] = q[3];
            pr[c] = q[4];
        }
}

/* Global sums of rho, j_x, j_y, e over the interior. */
void orc_sums(const orc_model *m, const orc_params *p, const double *f, double out[4])
{
    double a[4] = {0, 0, 0, 0};
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double fh[NQ];
            orc_moments(m, f + cell(p, i, j), fh);
            for (int k = 0; k < 4; ++k) a[k] += fh[k];
        }
    for (int k = 0; k < 4; ++k) out[k] = a[k];
}

/* ------------------------------------------------------------------------
 * Boundary nodes.  The paper sets f = f^eq of a macroscopic state on the
 * boundary nodes (Sect. V.A, V.B) and names how that state is found:
 * prescribed (Dirichlet), periodic, reflecting (normal velocity reversed),
 * linear extrapolation, and moving isothermal walls (Sect. V.D).  Here the
 * boundary nodes are one ghost layer outside the interior.
 *
 * Extrapolation takes q_g = 2 q_1 - q_2 on (rho, u1, u2, T) from the first
 * two interior nodes along the normal; if that leaves rho or T non-positive
 * the ghost takes q_1 instead.
 *
 * A side may switch rule at a moving point along it:
 * the rule is kind_lo where the node's along-side coordinate (cell-centred,
 * x = (i + 1/2) dx or y = (j + 1/2) dy) is <= split0 + split_rate * t, and
 * kind_hi beyond.  This expresses the Mach-reflection set-up (Sect. V.B).
 * ---------------------------------------------------------------------- */
static void side_state(const orc_model *m, const orc_params *p, const double *f, int sd,
                       int kind, const double st[4], int a, double out[NQ])
{
    /* a = along-side index; n1/n2 = first/second interior node along the normal */
    const int nx = p->nx, ny = p->ny;
    const double *n1, *n2;
    int normal; /* 0: x normal, 1: y normal */
    switch (sd) {
    case 0: n1 = f + cell(p, 0, a); n2 = f + cell(p, 1, a); normal = 0; break;
    case 1: n1 = f + cell(p, nx - 1, a); n2 = f + cell(p, nx - 2, a); normal = 0; break;
    case 2: n1 = f + cell(p, a, 0); n2 = f + cell(p, a, 1); normal = 1; break;
    default: n1 = f + cell(p, a, ny - 1); n2 = f + cell(p, a, ny - 2); normal = 1; break;
    }
    if (kind == ORC_PERIODIC) {
        const double *src;
        switch (sd) {
        case 0: src = f + cell(p, nx - 1, a); break;
        case 1: src = f + cell(p, 0, a); break;
        case 2: src = f + cell(p, a, ny - 1); break;
        default: src = f + cell(p, a, 0); break;
        }
        memcpy(out, src, sizeof(double) * NQ);
        return;
    }
    double q[4];
    if (kind == ORC_DIRICHLET) {
        for (int k = 0; k < 4; ++k) q[k] = st[k];
    } else {
        double q1[5], q2[5];
        orc_macro_of(m, n1, q1);
        if (kind == ORC_REFLECT) {
            for (int k = 0; k < 4; ++k) q[k] = q1[k];
            q[1 + normal] = -q1[1 + normal];
        } else if (kind == ORC_EXTRAPOLATE) {
            orc_macro_of(m, n2, q2);
            for (int k = 0; k < 4; ++k) q[k] = 2.0 * q1[k] - q2[k];
            if (!(q[0] > 0.0) || !(q[3] > 0.0))
                for (int k = 0; k < 4; ++k) q[k] = q1[k];
        } else { /* ORC_WALL */
            q[0] = q1[0];
            q[1] = st[1];
            q[2] = st[2];
            q[3] = st[3];
        }
    }
    orc_feq_velocity(m, q[0], q[1], q[2], q[3], out);
}

void orc_fill_ghosts(const orc_model *m, const orc_params *p, double *f, double t)
{
    for (int sd = 0; sd < 4; ++sd) {
        const orc_side *S = &p->side[sd];
        const int len = sd < 2 ? p->ny : p->nx;
        const double h = sd < 2 ? p->dy : p->dx;
        const double split = S->split0 + S->split_rate * t;
        for (int a = 0; a < len; ++a) {
            const double pos = (a + 0.5) * h;
            const int lo = pos <= split;
            double *g;
            switch (sd) {
            case 0: g = f + cell(p, -1, a); break;
            case 1: g = f + cell(p, p->nx, a); break;
            case 2: g = f + cell(p, a, -1); break;
            default: g = f + cell(p, a, p->ny); break;
            }
            side_state(m, p, f, sd, lo ? S->kind_lo : S->kind_hi, lo ? S->state_lo : S->state_hi,
                       a, g);
        }
    }
}

/* One time step: fill the boundary nodes of fin at time t, then update every
 * interior node into fout. */
/* ------------------------------------------------------------------------
 * Outflow through the sides (a budget for the conserved moments).  The
 * difference of Eq. (A.1b) along x is a difference of face values,
 *   dt [v d f/dx] = (dt/dx) (Phi(x + dx/2) - Phi(x - dx/2)),
 *   Phi(x + dx/2) = v (f(x) + f(x+dx)) / 2 - v^2 dt (f(x+dx) - f(x)) / (2 dx),
 * and likewise along y, so over the interior the sums of the conserved
 * moments m_1..m_4 (rho, j, e) change in one step by minus the face values
 * summed over the outer faces (the collision conserves them, Eq. 3).  Added
 * to out[side*4 + k]: the outflow of m_{k+1} through side (west, east,
 * south, north) in the step that starts from f (ghosts filled at t_n).
 * ---------------------------------------------------------------------- */
static double face_value(double v, double h, double dt, double f_lo, double f_hi)
{
    /* Phi between the node at the lower coordinate (f_lo) and the higher one */
    return v * (f_lo + f_hi) / 2.0 - v * v * dt * (f_hi - f_lo) / (2.0 * h);
}

void orc_face_outflow(const orc_model *m, const orc_params *p, const double *f, double out[16])
{
    const int nx = p->nx, ny = p->ny;
    const double dx = p->dx, dy = p->dy, dt = p->dt;
    for (int j = 0; j < ny; ++j) {
        const double *gw = f + cell(p, -1, j), *f0 = f + cell(p, 0, j);
        const double *fe = f + cell(p, nx - 1, j), *ge = f + cell(p, nx, j);
        for (int i = 0; i < NQ; ++i) {
            const double vx = m->v[i][0];
            if (vx == 0.0) continue;
            const double west = -(dt / dx) * face_value(vx, dx, dt, gw[i], f0[i]);
            const double east = (dt / dx) * face_value(vx, dx, dt, fe[i], ge[i]);
            for (int k = 0; k < 4; ++k) {
                out[0 * 4 + k] += m->M[k][i] * west;
                out[1 * 4 + k] += m->M[k][i] * east;
            }
        }
    }
    for (int a = 0; a < nx; ++a) {
        const double *gs = f + cell(p, a, -1), *f0 = f + cell(p, a, 0);
        const double *fn = f + cell(p, a, ny - 1), *gn = f + cell(p, a, ny);
        for (int i = 0; i < NQ; ++i) {
            const double vy = m->v[i][1];
            if (vy == 0.0) continue;
            const double south = -(dt / dy) * face_value(vy, dy, dt, gs[i], f0[i]);
            const double north = (dt / dy) * face_value(vy, dy, dt, fn[i], gn[i]);
            for (int k = 0; k < 4; ++k) {
                out[2 * 4 + k] += m->M[k][i] * south;
                out[3 * 4 + k] += m->M[k][i] * north;
            }
        }
    }
}

/* One step.  If outflow is not NULL the step's outflow through the sides is
 * added to it (see orc_face_outflow). */
void orc_step(const orc_model *m, const orc_params *p, double *fin, double *fout, double t,
              int nthreads, double *outflow)
{
    orc_fill_ghosts(m, p, fin, t);
    if (outflow) orc_face_outflow(m, p, fin, outflow);
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            orc_cell_update(m, p, fin + cell(p, i, j), fin + cell(p, i + 1, j),
                            fin + cell(p, i - 1, j), fin + cell(p, i, j + 1),
                            fin + cell(p, i, j - 1), fout + cell(p, i, j));
}

/* nsteps steps from step index step0 (time t = n dt at step n).  f holds the
 * state on entry and on return; work is a second buffer of the same size.
 * outflow (16 doubles, may be NULL) accumulates the outflow of every step. */
void orc_run(const orc_model *m, const orc_params *p, double *f, double *work, int64_t step0,
             int64_t nsteps, int nthreads, double *outflow)
{
    const size_t n = (size_t)(p->nx + 2) * (size_t)(p->ny + 2) * NQ;
    double *a = f, *b = work;
    for (int64_t k = 0; k < nsteps; ++k) {
        orc_step(m, p, a, b, (double)(step0 + k) * p->dt, nthreads, outflow);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, n * sizeof(double));
    /* leave the ghost layer of f describing the returned state */
    orc_fill_ghosts(m, p, f, (double)(step0 + nsteps) * p->dt);
}
