// Host side of the MRT finite-difference lattice Boltzmann library: the model
// constants (velocity set, M, its FP64 inverse, the factored FP32 transform),
// parameter validation, the context, the HIP-graph step loop, the step-kernel
// autotuner and the C ABI declared in include/mrtfd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "../../include/mrtfd.h"
#include "mrtfd_internal.h"

using namespace mrtfd;

namespace {

// ------------------------------------------------------------------ model

// Discrete velocities of Eq. (4), grouped (+-1 axes, +-6 axes, sqrt2
// diagonals, 3/sqrt2 diagonals), in the order printed in the rows of M.
void velocity_set(double v[NQ][2])
{
    const double ax[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    const double dg[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    const double scale[4] = {1.0, 6.0, std::sqrt(2.0), 3.0 / std::sqrt(2.0)};
    for (int g = 0; g < 4; ++g)
        for (int k = 0; k < 4; ++k) {
            const double(*dir)[2] = g < 2 ? ax : dg;
            v[4 * g + k][0] = scale[g] * dir[k][0];
            v[4 * g + k][1] = scale[g] * dir[k][1];
        }
}

// Row r of M evaluated at velocity (x, y): the polynomials of Eq. (5a)-(5p).
double m_row(int r, double x, double y)
{
    const double q = x * x + y * y, c2 = x * x - y * y, s2 = x * y;
    const double c3 = x * (x * x - 3 * y * y), s3 = y * (3 * x * x - y * y);
    switch (r) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return 0.5 * q;
    case 4: return c2;
    case 5: return s2;
    case 6: return 0.5 * q * x;
    case 7: return 0.5 * q * y;
    case 8: return c3;
    case 9: return s3;
    case 10: return 0.25 * q * q;
    case 11: return c2 * c2 - 4 * s2 * s2;  // x^4 - 6 x^2 y^2 + y^4
    case 12: return q * c2;
    case 13: return q * s2;
    case 14: return q * c3;
    default: return q * s3;
    }
}

// LU factorisation with partial pivoting, then n solves for the columns of
// the inverse.  Returns false for a singular matrix.
bool lu_inverse(int n, const double *A, double *Ainv)
{
    std::vector<double> a(A, A + n * n);
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int r = k + 1; r < n; ++r)
            if (std::fabs(a[r * n + k]) > std::fabs(a[p * n + k])) p = r;
        if (a[p * n + k] == 0.0) return false;
        piv[k] = p;
        if (p != k)
            for (int c = 0; c < n; ++c) std::swap(a[k * n + c], a[p * n + c]);
        for (int r = k + 1; r < n; ++r) {
            a[r * n + k] /= a[k * n + k];
            for (int c = k + 1; c < n; ++c) a[r * n + c] -= a[r * n + k] * a[k * n + c];
        }
    }
    for (int col = 0; col < n; ++col) {
        std::vector<double> b(n, 0.0);
        b[col] = 1.0;
        for (int k = 0; k < n; ++k)
            if (piv[k] != k) std::swap(b[k], b[piv[k]]);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < r; ++c) b[r] -= a[r * n + c] * b[c];
        for (int r = n - 1; r >= 0; --r) {
            for (int c = r + 1; c < n; ++c) b[r] -= a[r * n + c] * b[c];
            b[r] /= a[r * n + r];
        }
        for (int r = 0; r < n; ++r) Ainv[r * n + col] = b[r];
    }
    return true;
}

struct Model {
    double v[NQ][2];
    double M[NQ][NQ], Minv[NQ][NQ];
    // Butterfly P (u = P f, u = [A0..3, X0..3, Y0..3, Q0..3]), B = M P^-1 and
    // D B^-1 = D P M^-1 with D the butterfly scales (inverse butterfly = adds).
    double B[NQ][NQ], DBinv[NQ][NQ];
    bool ok = false;
    char why[160] = {0};
};

Model build_model()
{
    Model m;
    velocity_set(m.v);
    for (int r = 0; r < NQ; ++r)
        for (int i = 0; i < NQ; ++i) m.M[r][i] = m_row(r, m.v[i][0], m.v[i][1]);
    if (!lu_inverse(NQ, &m.M[0][0], &m.Minv[0][0])) {
        std::snprintf(m.why, sizeof m.why, "M is singular");
        return m;
    }
    double P[NQ][NQ] = {{0}}, Pinv[NQ][NQ];
    const int sx_axis[4] = {1, 0, -1, 0}, sy_axis[4] = {0, 1, 0, -1};
    const int sx_diag[4] = {1, -1, -1, 1}, sy_diag[4] = {1, 1, -1, -1};
    const int sq[4] = {1, -1, 1, -1};
    for (int g = 0; g < 4; ++g)
        for (int k = 0; k < 4; ++k) {
            const int c = 4 * g + k;
            P[g][c] = 1.0;
            P[4 + g][c] = g < 2 ? sx_axis[k] : sx_diag[k];
            P[8 + g][c] = g < 2 ? sy_axis[k] : sy_diag[k];
            P[12 + g][c] = sq[k];
        }
    if (!lu_inverse(NQ, &P[0][0], &Pinv[0][0])) {
        std::snprintf(m.why, sizeof m.why, "butterfly is singular");
        return m;
    }
    // D: axis groups A,Q /4 and X,Y /2; diagonal groups all /4.
    double D[NQ];
    for (int g = 0; g < 4; ++g) {
        D[g] = D[12 + g] = 0.25;
        D[4 + g] = D[8 + g] = g < 2 ? 0.5 : 0.25;
    }
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < NQ; ++c) {
            double b = 0.0, bi = 0.0;
            for (int k = 0; k < NQ; ++k) {
                b += m.M[r][k] * Pinv[k][c];
                bi += P[r][k] * m.Minv[k][c];
            }
            m.B[r][c] = b;
            m.DBinv[r][c] = D[r] * bi;
        }
    // The block structure the kernels rely on: check that everything outside
    // the blocks vanishes, and that the adds-only inverse butterfly applied
    // to D B^-1 gives back M^-1.
    auto block_of_moment = [](int k) {
        switch (k) {
        case 0: case 3: case 10: case 11: return 0;
        case 1: case 6: case 8: case 14: return 1;
        case 2: case 7: case 9: case 15: return 2;
        case 4: case 12: return 3;
        default: return 4;  // 5, 13
        }
    };
    auto block_of_comb = [](int c) {
        if (c < 4) return 0;
        if (c < 8) return 1;
        if (c < 12) return 2;
        return c < 14 ? 3 : 4;
    };
    double worst = 0.0;
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < NQ; ++c) {
            if (block_of_moment(r) != block_of_comb(c))
                worst = std::max(worst, std::fabs(m.B[r][c]) / 7776.0);
            if (block_of_comb(r) != block_of_moment(c)) worst = std::max(worst, std::fabs(m.DBinv[r][c]));
        }
    double E[NQ][NQ] = {{0}};  // inverse butterfly as adds (group_inv in the kernels)
    for (int g = 0; g < 4; ++g) {
        const int a = g, x = 4 + g, y = 8 + g, q = 12 + g, b = 4 * g;
        E[b + 0][a] = 1; E[b + 0][q] = 1;
        E[b + 2][a] = 1; E[b + 2][q] = 1;
        E[b + 1][a] = 1; E[b + 1][q] = -1;
        E[b + 3][a] = 1; E[b + 3][q] = -1;
        if (g < 2) {
            E[b + 0][x] = 1; E[b + 2][x] = -1; E[b + 1][y] = 1; E[b + 3][y] = -1;
        } else {
            E[b + 0][x] = 1; E[b + 0][y] = 1;
            E[b + 2][x] = -1; E[b + 2][y] = -1;
            E[b + 1][x] = -1; E[b + 1][y] = 1;
            E[b + 3][x] = 1; E[b + 3][y] = -1;
        }
    }
    for (int r = 0; r < NQ; ++r)
        for (int c = 0; c < NQ; ++c) {
            double acc = 0.0;
            for (int k = 0; k < NQ; ++k) acc += E[r][k] * m.DBinv[k][c];
            worst = std::max(worst, std::fabs(acc - m.Minv[r][c]));
        }
    if (worst > 1e-12) {
        std::snprintf(m.why, sizeof m.why, "transform structure check failed (%.3g)", worst);
        return m;
    }
    m.ok = true;
    return m;
}

const Model &model()
{
    static const Model m = build_model();
    return m;
}

// f^eq = M^-1 f-hat^eq of a macroscopic state, FP64 (Dirichlet boundary states).
void feq_host(const Model &m, double rho, double ux, double uy, double T, double out[NQ])
{
    const double jx = rho * ux, jy = rho * uy, e = rho * (T + 0.5 * (ux * ux + uy * uy));
    const double P = rho * T, j2 = jx * jx + jy * jy;
    double h[NQ] = {rho, jx, jy, e,
                    (jx * jx - jy * jy) / rho, jx * jy / rho, (e + P) * jx / rho, (e + P) * jy / rho,
                    (jx * jx - 3 * jy * jy) * jx / (rho * rho), (3 * jx * jx - jy * jy) * jy / (rho * rho),
                    2 * e * e / rho - j2 * j2 / (4 * rho * rho * rho), 0.0,
                    (6 * rho * e - 2 * j2) * (jx * jx - jy * jy) / (rho * rho * rho),
                    (6 * rho * e - 2 * j2) * jx * jy / (rho * rho * rho), 0.0, 0.0};
    for (int i = 0; i < NQ; ++i) {
        double a = 0.0;
        for (int k = 0; k < NQ; ++k) a += m.Minv[i][k] * h[k];
        out[i] = a;
    }
}

// The reference state at rest (rho0, T0), rounded to FP32 as the kernels
// hold it; (0, 0) when none is set.
void ref_state(const mrtfd_params &p, double &rho0, double &T0)
{
    rho0 = p.ref_rho > 0 ? (double)(float)p.ref_rho : 0.0;
    T0 = p.ref_rho > 0 ? (double)(float)p.ref_T : 0.0;
}

// f_ref = M^-1 f-hat^eq(rho0, 0, 0, rho0 T0) in FP64; zeros without a reference.
void ref_populations(const Model &m, const mrtfd_params &p, double out[NQ])
{
    double rho0, T0;
    ref_state(p, rho0, T0);
    if (rho0 > 0)
        feq_host(m, rho0, 0.0, 0.0, T0, out);
    else
        for (int q = 0; q < NQ; ++q) out[q] = 0.0;
}

// The step constants in the stored precision (FP64 products, then rounded).
template <class Real>
void fill_consts(const Model &m, const mrtfd_params &p, ConstsT<Real> &K)
{
    std::memset(&K, 0, sizeof K);
    const int r0[4] = {0, 3, 10, 11}, rx[4] = {1, 6, 8, 14}, ry[4] = {2, 7, 9, 15};
    const int rqa[2] = {4, 12}, rqd[2] = {5, 13};
    for (int a = 0; a < 4; ++a)
        for (int g = 0; g < 4; ++g) {
            K.f0[a][g] = (Real)m.B[r0[a]][g];
            K.fx[a][g] = (Real)m.B[rx[a]][4 + g];
            K.fy[a][g] = (Real)m.B[ry[a]][8 + g];
            K.i0[g][a] = (Real)m.DBinv[g][r0[a]];
            K.ix[g][a] = (Real)m.DBinv[4 + g][rx[a]];
            K.iy[g][a] = (Real)m.DBinv[8 + g][ry[a]];
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            K.fqa[a][b] = (Real)m.B[rqa[a]][12 + b];
            K.fqd[a][b] = (Real)m.B[rqd[a]][14 + b];
            K.iqa[a][b] = (Real)m.DBinv[12 + a][rqa[b]];
            K.iqd[a][b] = (Real)m.DBinv[14 + a][rqd[b]];
        }
    // collision columns: D B^-1 scaled by dt s_k (FP64 product, then rounded)
    const double dt = p.dt;
    auto cs = [&](int row, int k) { return (Real)(m.DBinv[row][k] * dt * p.s[k]); };
    const int k0[2] = {10, 11}, kx[3] = {6, 8, 14}, ky[3] = {7, 9, 15};
    for (int g = 0; g < 4; ++g) {
        for (int a = 0; a < 2; ++a) K.c0[g][a] = cs(g, k0[a]);
        for (int a = 0; a < 3; ++a) {
            K.cx[g][a] = cs(4 + g, kx[a]);
            K.cy[g][a] = cs(8 + g, ky[a]);
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            K.cqa[a][b] = cs(12 + a, rqa[b]);
            K.cqd[a][b] = cs(14 + a, rqd[b]);
        }
    for (int q = 0; q < NQ; ++q) {
        const double a = m.v[q][0] * dt / p.dx, b = m.v[q][1] * dt / p.dy;
        K.lw[q][0] = (Real)(0.5 * (a * a - a));
        K.lw[q][1] = (Real)(0.5 * (a * a + a));
        K.lw[q][2] = (Real)(0.5 * (b * b - b));
        K.lw[q][3] = (Real)(0.5 * (b * b + b));
    }
    double rho0, T0;
    ref_state(p, rho0, T0);
    K.rho0 = (Real)rho0;
    K.T0 = (Real)T0;
    K.e0 = (Real)(rho0 * T0);
    K.Te0 = (Real)(T0 * rho0 * T0);
}

// BF16 bits of an FP32 value, round to nearest even (as the kernels do).
unsigned short bf16_of(float x)
{
    unsigned u;
    std::memcpy(&u, &x, 4);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
double bf16_value(unsigned short b)
{
    const unsigned u = (unsigned)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Block table (Bf3Ops) from the FP32 constants.  Forward blocks 0-3: their
// entries are small dyadic numbers, or sqrt 2 times one in the diagonal
// groups' columns (2, 3) of fx and fy, which the table holds divided by
// sqrt 2; each must then be exact in BF16 (false if not).  Back-map blocks
// 4-7: each FP32 entry as three BF16 parts (round to nearest even, then the
// remainders likewise), which add up to it exactly.
bool fill_bf3(const Consts &K, Bf3Ops &out)
{
    double W[8][4][4] = {};
    for (int i = 0; i < 4; ++i)
        for (int c = 0; c < 4; ++c) {
            const double r = c >= 2 ? 1.0 / std::sqrt(2.0) : 1.0;
            W[0][i][c] = K.f0[i][c];
            W[1][i][c] = K.fx[i][c] * r;
            W[2][i][c] = K.fy[i][c] * r;
        }
    for (int i = 0; i < 2; ++i) {
        W[3][i][0] = K.fqa[i][0];      // m5, m13 over Q0, Q1
        W[3][i][1] = K.fqa[i][1];
        W[3][2 + i][2] = K.fqd[i][0];  // m6, m14 over Q2, Q3
        W[3][2 + i][3] = K.fqd[i][1];
        W[7][i][0] = K.cqa[i][0];      // Q0, Q1 over m5, m13
        W[7][i][1] = K.cqa[i][1];
        W[7][2 + i][2] = K.cqd[i][0];  // Q2, Q3 over m6, m14
        W[7][2 + i][3] = K.cqd[i][1];
    }
    for (int g = 0; g < 4; ++g) {
        W[4][g][0] = K.c0[g][0];
        W[4][g][1] = K.c0[g][1];
        for (int c = 0; c < 3; ++c) {
            W[5][g][c] = K.cx[g][c];
            W[6][g][c] = K.cy[g][c];
        }
    }
    std::memset(&out, 0, sizeof out);
    for (int b = 0; b < 8; ++b)
        for (int i = 0; i < 4; ++i) {
            unsigned short hi[4], mid[4] = {}, lo[4] = {};
            for (int c = 0; c < 4; ++c) {
                const double w = W[b][i][c];
                hi[c] = bf16_of((float)w);
                if (b < 4) {
                    // FP32 constants: exact up to their own rounding
                    if (std::fabs(w - bf16_value(hi[c])) > 0x1p-22 * std::fabs(w)) return false;
                    continue;
                }
                const float r = (float)(w - bf16_value(hi[c]));  // exact: w is an FP32 value
                mid[c] = bf16_of(r);
                lo[c] = bf16_of((float)(r - bf16_value(mid[c])));
                if (bf16_value(hi[c]) + bf16_value(mid[c]) + bf16_value(lo[c]) != w) return false;
            }
            out.w[b][i] = make_uint4(hi[0] | (unsigned)hi[1] << 16, hi[2] | (unsigned)hi[3] << 16,
                                     mid[0] | (unsigned)mid[1] << 16, mid[2] | (unsigned)mid[3] << 16);
            if (b >= 4)
                out.w[b + 4][i] = make_uint4(lo[0] | (unsigned)lo[1] << 16, lo[2] | (unsigned)lo[3] << 16, 0u, 0u);
        }
    return true;
}

// Boundary description of the step kernels in the stored precision: per side
// its rule pair and switch point, the states as deviations from the
// reference state (rho - rho0, u1, u2, T - T0) and the Dirichlet equilibria
// as f^eq - f_ref, both formed in FP64 and then rounded.  kcopy, gcopy and
// fcopy are the workspace addresses of the device copies of the constants,
// of this struct and of the outflow coefficients.
template <class Real>
void fill_ghosts(const Model &m, const mrtfd_params &p, const double (&fref)[NQ], char *kcopy,
                 char *gcopy, char *fcopy, GhostsT<Real> &G)
{
    double rho0, T0;
    ref_state(p, rho0, T0);
    G.dt = p.dt;
    G.kd = reinterpret_cast<const ConstsT<Real> *>(kcopy);
    G.gd = reinterpret_cast<const GhostsT<Real> *>(gcopy);
    G.fd = reinterpret_cast<const FluxCoef *>(fcopy);
    G.per_x = p.side[0].kind_lo == MRTFD_BC_PERIODIC;
    G.per_y = p.side[2].kind_lo == MRTFD_BC_PERIODIC;
    for (int s = 0; s < 4; ++s) {
        const mrtfd_side &S = p.side[s];
        GhostSideT<Real> &g = G.side[s];
        g.kind_lo = S.kind_lo;
        g.kind_hi = S.kind_hi;
        g.split0 = S.split0;
        g.split_rate = S.split_rate;
        g.h = s < 2 ? p.dy : p.dx;
        const double off[4] = {rho0, 0.0, 0.0, T0};
        for (int k = 0; k < 4; ++k) {
            g.st_lo[k] = (Real)(S.state_lo[k] - off[k]);
            g.st_hi[k] = (Real)(S.state_hi[k] - off[k]);
        }
        double fe[NQ];
        for (int q = 0; q < NQ; ++q) g.feq_lo[q] = g.feq_hi[q] = Real(0);
        if (S.kind_lo == MRTFD_BC_DIRICHLET) {
            feq_host(m, S.state_lo[0], S.state_lo[1], S.state_lo[2], S.state_lo[3], fe);
            for (int q = 0; q < NQ; ++q) g.feq_lo[q] = (Real)(fe[q] - fref[q]);
        }
        if (S.kind_hi == MRTFD_BC_DIRICHLET) {
            feq_host(m, S.state_hi[0], S.state_hi[1], S.state_hi[2], S.state_hi[3], fe);
            for (int q = 0; q < NQ; ++q) g.feq_hi[q] = (Real)(fe[q] - fref[q]);
        }
    }
}

// ------------------------------------------------------- stability screen

// d f-hat^eq / d (rho, j_x, j_y, e) by complex steps (Squire and Trapp,
// 1998): for an analytic h, Im h(x + i eps e_c) / eps = dh/dx_c with no
// difference of nearby values, so the result is exact up to rounding.
void feq_jacobian(double rho, double jx, double jy, double e, double J[NQ][4])
{
    const double eps = 1e-30;
    for (int c = 0; c < 4; ++c) {
        std::complex<double> x[4] = {rho, jx, jy, e};
        x[c] += std::complex<double>(0.0, eps);
        std::complex<double> h[NQ];
        feq_of_conserved(x[0], x[1], x[2], x[3], h);
        for (int k = 0; k < NQ; ++k) J[k][c] = h[k].imag() / eps;
    }
}

// The screen's phase-independent part at a uniform state (rho, u1, u2, T):
// C = dt M^-1 S (M - J M_c), J the Jacobian above and M_c the conserved rows
// of M (the chain rule of Sect. IV through rho, j, e); and the Lax-Wendroff
// weights a_i, b_i.
void screen_coef(const Model &m, const mrtfd_params &p, const double state[4], ScreenCoef &S)
{
    const double rho = state[0], ux = state[1], uy = state[2], T = state[3];
    double J[NQ][4];
    feq_jacobian(rho, rho * ux, rho * uy, rho * (T + 0.5 * (ux * ux + uy * uy)), J);
    double D[NQ][NQ];
    for (int k = 0; k < NQ; ++k)
        for (int i = 0; i < NQ; ++i) {
            double a = m.M[k][i];
            for (int c = 0; c < 4; ++c) a -= J[k][c] * m.M[c][i];
            D[k][i] = a;
        }
    for (int a = 0; a < NQ; ++a)
        for (int i = 0; i < NQ; ++i) {
            double acc = 0.0;
            for (int k = 0; k < NQ; ++k) acc += m.Minv[a][k] * p.s[k] * D[k][i];
            S.C[a][i] = p.dt * acc;
        }
    for (int q = 0; q < NQ; ++q) {
        S.a[q] = m.v[q][0] * p.dt / p.dx;
        S.b[q] = m.v[q][1] * p.dt / p.dy;
    }
}

// --------------------------------------------------------------- validation

int check(const mrtfd_params *p, char *msg, size_t len)
{
    auto fail = [&](int code, const char *fmt, ...) {
        if (msg && len) {
            va_list ap;
            va_start(ap, fmt);
            std::vsnprintf(msg, len, fmt, ap);
            va_end(ap);
        }
        return code;
    };
    if (!p) return fail(MRTFD_ERR_ARG, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(MRTFD_ERR_ARG, "nx and ny must be >= 3 (got %d, %d)", p->nx, p->ny);
    if ((long long)p->nx * p->ny > (1LL << 31))
        return fail(MRTFD_ERR_ARG, "grid of %lld nodes is too large", (long long)p->nx * p->ny);
    {
        // the row and matrix-core kernels address one copy of f with 32-bit
        // byte offsets: (ny + 2) rows of 16 x pitch values must stay below 4 GiB
        const long long pitch = ((long long)p->nx + 65 + 63) / 64 * 64;
        const long long esize = p->precision == MRTFD_FP64 ? 8 : 4;
        const long long bytes = esize * NQ * pitch * ((long long)p->ny + 2);
        if (bytes >= (1LL << 32) && p->kernel != MRTFD_KERNEL_SIMPLE)
            return fail(MRTFD_ERR_ARG,
                        "grid %d x %d needs %lld bytes per copy of f: above 4 GiB only "
                        "MRTFD_KERNEL_SIMPLE runs it", p->nx, p->ny, bytes);
        if (bytes >= (1LL << 32) && p->precision == MRTFD_BF16X3)
            return fail(MRTFD_ERR_ARG, "grids above 4 GiB per copy of f run in FP32 or FP64");
    }
    if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0) || !std::isfinite(p->dx) ||
        !std::isfinite(p->dy) || !std::isfinite(p->dt))
        return fail(MRTFD_ERR_ARG, "dx, dy, dt must be positive and finite");
    for (int k = 4; k < NQ; ++k) {
        if (!(p->s[k] >= 0) || !std::isfinite(p->s[k]))
            return fail(MRTFD_ERR_ARG, "s_%d must be finite and >= 0", k + 1);
        if (p->dt * p->s[k] > 1.0 + 1e-12)
            return fail(MRTFD_ERR_UNSTABLE, "dt * s_%d = %g exceeds 1", k + 1, p->dt * p->s[k]);
    }
    const double cfl = 6.0 * p->dt / std::min(p->dx, p->dy);
    if (cfl > 1.0) return fail(MRTFD_ERR_UNSTABLE, "Courant number 6 dt / min(dx,dy) = %g exceeds 1", cfl);
    if (p->precision != MRTFD_FP32 && p->precision != MRTFD_BF16X3 && p->precision != MRTFD_FP64)
        return fail(MRTFD_ERR_ARG, "unknown precision mode %d", p->precision);
    if (p->precision == MRTFD_FP64 && p->rows == 2)
        return fail(MRTFD_ERR_ARG, "MRTFD_FP64 runs the rows kernel at one row per wave (rows 0 or 1)");
    if (p->collision != MRTFD_COLLISION_MRT && p->collision != MRTFD_COLLISION_SRT)
        return fail(MRTFD_ERR_ARG, "unknown collision %d", p->collision);
    if (p->collision == MRTFD_COLLISION_SRT) {
        for (int k = 5; k < NQ; ++k)
            if (p->s[k] != p->s[4])
                return fail(MRTFD_ERR_ARG, "single relaxation time needs s_6..s_16 equal to s_5");
    }
    if (p->layout != MRTFD_LAYOUT_ROWS && p->layout != MRTFD_LAYOUT_PLANES &&
        p->layout != MRTFD_LAYOUT_TILES)
        return fail(MRTFD_ERR_ARG, "unknown layout %d", p->layout);
    if (p->kernel != MRTFD_KERNEL_AUTO && p->kernel != MRTFD_KERNEL_SIMPLE &&
        p->kernel != MRTFD_KERNEL_ROWS)
        return fail(MRTFD_ERR_ARG, "unknown kernel %d", p->kernel);
    if (p->rows != 0 && p->rows != 1 && p->rows != 2)
        return fail(MRTFD_ERR_ARG, "rows must be 0, 1 or 2");
    if (p->flux_budget != 0 && p->flux_budget != 1)
        return fail(MRTFD_ERR_ARG, "flux_budget must be 0 or 1");
    if (p->graph_steps < 0 || (p->graph_steps % 2) != 0 || p->graph_steps > 4096)
        return fail(MRTFD_ERR_ARG, "graph_steps must be even, in [0, 4096]");
    if (!std::isfinite(p->ref_rho) || !std::isfinite(p->ref_T) || p->ref_rho < 0 || p->ref_T < 0 ||
        ((p->ref_rho > 0) != (p->ref_T > 0)) ||
        (p->ref_rho > 0 && (!((float)p->ref_rho > 0.f) || !((float)p->ref_T > 0.f) ||
                            !std::isfinite((float)p->ref_rho) || !std::isfinite((float)p->ref_T))))
        return fail(MRTFD_ERR_ARG, "reference state: ref_rho and ref_T both > 0 (FP32 range), or both 0");
    for (int s = 0; s < 4; ++s) {
        const mrtfd_side &S = p->side[s];
        for (int part = 0; part < 2; ++part) {
            const int kind = part ? S.kind_hi : S.kind_lo;
            const double *st = part ? S.state_hi : S.state_lo;
            if (kind < MRTFD_BC_PERIODIC || kind > MRTFD_BC_WALL)
                return fail(MRTFD_ERR_ARG, "side %d: unknown rule %d", s, kind);
            if (kind == MRTFD_BC_PERIODIC) {
                const mrtfd_side &O = p->side[s ^ 1];
                if (O.kind_lo != MRTFD_BC_PERIODIC || O.kind_hi != MRTFD_BC_PERIODIC ||
                    S.kind_lo != MRTFD_BC_PERIODIC || S.kind_hi != MRTFD_BC_PERIODIC)
                    return fail(MRTFD_ERR_ARG, "side %d: periodic needs the opposite side periodic", s);
            }
            if (kind == MRTFD_BC_DIRICHLET && (!(st[0] > 0) || !(st[3] > 0)))
                return fail(MRTFD_ERR_ARG, "side %d: Dirichlet state needs rho > 0 and T > 0", s);
            if (kind == MRTFD_BC_WALL && !(st[3] > 0))
                return fail(MRTFD_ERR_ARG, "side %d: wall temperature must be > 0", s);
            for (int c = 0; c < 4; ++c)
                if (!std::isfinite(st[c])) return fail(MRTFD_ERR_ARG, "side %d: state is not finite", s);
        }
        if (std::isnan(S.split0) || !std::isfinite(S.split_rate))
            return fail(MRTFD_ERR_ARG, "side %d: bad split point", s);
    }
    if (msg && len) msg[0] = 0;
    return MRTFD_OK;
}

Field make_field(const mrtfd_params &p)
{
    Field F;
    F.nx = p.nx;
    F.ny = p.ny;
    F.xoff = 64;
    F.pitch = ((F.xoff + p.nx + 1 + 63) / 64) * 64;
    F.total = (long long)NQ * F.pitch * (p.ny + 2);
    F.tstride = 64;
    if (p.layout == MRTFD_LAYOUT_PLANES) {
        F.qstride = (long long)F.pitch * (p.ny + 2);
        F.jstride = F.pitch;
    } else if (p.layout == MRTFD_LAYOUT_TILES) {
        F.qstride = 64;
        F.jstride = (long long)NQ * F.pitch;
        F.tstride = 64LL * NQ;
    } else {
        F.qstride = F.pitch;
        F.jstride = (long long)NQ * F.pitch;
    }
    return F;
}

struct Layout {
    size_t fA, fB, partials, sums, step, flag, bf3, kcopy, gcopy, fcopy, flux, outflow, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout(const mrtfd_params &p)
{
    const Field F = make_field(p);
    Layout L;
    const size_t esize = p.precision == MRTFD_FP64 ? sizeof(double) : sizeof(float);
    const size_t fbytes = align256((size_t)F.total * esize);
    L.fA = 0;
    L.fB = L.fA + fbytes;
    L.partials = L.fB + fbytes;
    L.sums = L.partials + align256(1024 * 4 * sizeof(double));
    L.step = L.sums + 256;
    L.flag = L.step + 256;
    L.bf3 = L.flag + 256;
    L.kcopy = L.bf3 + align256(sizeof(Bf3Ops));
    L.gcopy = L.kcopy + align256(sizeof(Consts64));  // room for either precision
    L.fcopy = L.gcopy + align256(sizeof(Ghosts64));
    L.flux = L.fcopy + align256(sizeof(FluxCoef));
    L.outflow = L.flux + (p.flux_budget ? align256(2 * ((size_t)p.nx + p.ny) * 4 * sizeof(double)) : 0);
    L.total = L.outflow + 256;
    return L;
}

// ----------------------------------------------------------- autotune cache

struct TuneKey {
    int nx, ny, layout, kernel, rows, precision, budget;
    bool operator<(const TuneKey &o) const
    {
        if (nx != o.nx) return nx < o.nx;
        if (ny != o.ny) return ny < o.ny;
        if (layout != o.layout) return layout < o.layout;
        if (kernel != o.kernel) return kernel < o.kernel;
        if (rows != o.rows) return rows < o.rows;
        if (precision != o.precision) return precision < o.precision;
        return budget < o.budget;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

}  // namespace

// ------------------------------------------------------------------ context

struct mrtfd_ctx {
    mrtfd_params p;
    Field F;
    Consts K;
    Ghosts G;
    Consts64 K64;                // FP64 mode: constants and boundary states in FP64
    Ghosts64 G64;
    SumW W;
    Layout L;
    char *ws = nullptr;
    float *f[2] = {nullptr, nullptr};      // the two copies of the stored values (FP32)
    double *f64[2] = {nullptr, nullptr};   // the same copies in the FP64 mode
    double *partials = nullptr, *sums = nullptr;
    long long *d_step = nullptr;
    int *d_flag = nullptr;
    Bf3Ops *d_bf3 = nullptr;      // device copy of the split-BF16 block table
    Bf3Ops h_bf3;
    double *flux = nullptr, *outflow = nullptr;  // outflow budget slots and totals
    double *scratch = nullptr;   // this device's library scratch (mrtfd_sums_noalloc)
    FluxCoef FC;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    // outflow budget: its kernel runs on `side`, beside the step kernel that
    // reads the same state (fork and join by the two events)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int device = 0;
    int cur = 0;                 // which copy holds the state
    long long step = 0;
    double fref[NQ] = {0};       // f_ref (FP64) of the reference state, zeros if none
    double ref_out[4][4] = {{0}};// outflow of f_ref per side node and step
    long long budget_steps = 0;  // steps added to the outflow budget since its reset
    bool initialised = false;
    int kernel = 0, seg = 0;     // step kernel in use and its rows per wave
    bool tuned = false;          // kernel/seg final (explicit, cached or timed)
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by starting copy
    char err[512] = {0};
};

namespace {

int set_err(mrtfd_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return set_err(ctx, MRTFD_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// The rows kernel at one row per wave carries the outflow budget in its own
// grid: the budget's FP64 path adds no register pressure to its interior
// path there.  At two rows per wave (already at the 128-register cap) it
// would, so that variant, like the other step kernels, gets the budget from
// k_face_flux on the side stream (enqueue_steps).  Trials of the autotuner
// run with the budget as configured, so the choice between the two prices
// it in.
bool budget_fused(const mrtfd_ctx *c)
{
    return c->p.flux_budget && (c->kernel == MRTFD_KERNEL_ROWS || c->kernel == MRTFD_KERNEL_MFMA) &&
           (c->seg & 15) == 1;
}

bool is64(const mrtfd_ctx *c) { return c->p.precision == MRTFD_FP64; }

// One step from copy a to copy a ^ 1.
hipError_t launch_step(mrtfd_ctx *c, int a, int k, hipStream_t s)
{
    if (is64(c)) {
        if (c->kernel == MRTFD_KERNEL_SIMPLE)
            return launch_step_simple(c->F, c->K64, c->G64, c->f64[a], c->f64[a ^ 1], c->d_step, k, s);
        return launch_step_rows(c->F, c->K64, c->G64, c->f64[a], c->f64[a ^ 1], c->seg & 15,
                                (c->seg >> 4) & 1, (c->seg >> 5) & 1, c->d_step, k, s,
                                budget_fused(c) ? c->flux : nullptr);
    }
    const float *fin = c->f[a];
    float *fout = c->f[a ^ 1];
    if (c->kernel == MRTFD_KERNEL_SIMPLE)
        return launch_step_simple(c->F, c->K, c->G, fin, fout, c->d_step, k, s);
    // the row kernels; with MRTFD_KERNEL_MFMA their split-BF16 variant
    return launch_step_rows(c->F, c->K, c->G, fin, fout, c->seg & 15, (c->seg >> 4) & 1,
                            (c->seg >> 5) & 1, c->d_step, k, s, budget_fused(c) ? c->flux : nullptr,
                            c->kernel == MRTFD_KERNEL_MFMA ? c->d_bf3 : nullptr);
}

// Enqueue n steps starting from copy `start`, then advance the device clock.
// With the outflow budget on, step k's budget kernel runs on the side stream
// concurrently with step k's update (both only read copy a), and step k + 1
// waits for both.  Under graph capture the side stream joins the capture
// through the fork event and is joined back before the capture ends.
hipError_t enqueue_steps(mrtfd_ctx *c, int start, int n, hipStream_t s)
{
    int a = start;
    for (int k = 0; k < n; ++k) {
        hipError_t e = hipSuccess;
        const bool side = c->p.flux_budget && !budget_fused(c);
        if (side) {
            e = hipEventRecord(c->ev_fork, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_fork, 0);
            if (e == hipSuccess)
                e = is64(c) ? launch_face_flux(c->F, c->K64, c->G64, c->FC, c->f64[a], c->flux, c->d_step,
                                               k, c->side)
                            : launch_face_flux(c->F, c->K, c->G, c->FC, c->f[a], c->flux, c->d_step, k,
                                               c->side);
            if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->side);
        }
        if (e == hipSuccess) e = launch_step(c, a, k, s);
        if (e == hipSuccess && side) e = hipStreamWaitEvent(s, c->ev_join, 0);
        if (e != hipSuccess) return e;
        a ^= 1;
    }
    return launch_counter_add(c->d_step, n, s);
}

void drop_graphs(mrtfd_ctx *c)
{
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) {
            (void)hipGraphExecDestroy(c->graph[k]);
            c->graph[k] = nullptr;
        }
}

// Debugging aid: with MRTFD_POISON_PADDING=1 in the environment at create,
// the copies of f start as NaN instead of zero, so that any read of a node
// outside the interior (the ring and the padding columns) shows in results.
bool poison_padding()
{
    const char *v = std::getenv("MRTFD_POISON_PADDING");
    return v && v[0] == '1' && v[1] == 0;
}

// Graphs, private streams and events, then the context itself.
void release(mrtfd_ctx *c)
{
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    delete c;
}

int build_graph(mrtfd_ctx *c, int start)
{
    if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_steps(c, start, c->p.graph_steps, c->cap);
    hipError_t e2 = hipStreamEndCapture(c->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return set_err(c, MRTFD_ERR_HIP, "graph capture failed: %s",
                       hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_err(c, MRTFD_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    c->graph[start] = ex;
    return MRTFD_OK;
}

// Advance the state by n direct launches (no graph).
hipError_t direct_steps(mrtfd_ctx *c, long long n)
{
    while (n > 0) {
        const int k = (int)std::min<long long>(n, 1 << 20);
        hipError_t e = enqueue_steps(c, c->cur, k, c->stream);
        if (e != hipSuccess) return e;
        if (k & 1) c->cur ^= 1;
        c->step += k;
        n -= k;
    }
    return hipSuccess;
}

// Pick the step kernel by timing each candidate on steps of the run itself.
// Every variant computes the same bits, so trial steps are ordinary steps;
// and timing them in the real alternation between the two copies sees the
// caches as a long run does (repeated launches on one input would not: the
// output of streaming stores, which bypass the last-level cache, is then
// never read back).  The candidates are timed in two passes and each keeps
// its faster time: the first steps of a run, and the first steps in a new
// tile order, run up to about a tenth slower than later ones, which biases a
// single pass against whichever candidates come early or change the order.
// Uses up to `avail` steps and reports how many it took in *taken.  When
// `avail` is too short for a fair trial the default variant stays in place
// and tuning waits for a longer call.
int autotune(mrtfd_ctx *c, long long avail, long long *taken)
{
    *taken = 0;
    if (c->tuned) return MRTFD_OK;
    const TuneKey key{c->p.nx, c->p.ny, c->p.layout, c->p.kernel, c->p.rows, c->p.precision,
                       c->p.flux_budget};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            const bool changed = c->kernel != it->second.first || c->seg != it->second.second;
            c->kernel = it->second.first;
            c->seg = it->second.second;
            c->tuned = true;
            // graphs captured before (a call too short to tune) hold the old
            // variant; they are rebuilt on the next replay
            if (changed) {
                HIPCHK(c, hipStreamSynchronize(c->stream));
                drop_graphs(c);
            }
            return MRTFD_OK;
        }
    }
    std::vector<std::pair<int, int>> cands;
    // second: rows per wave, (bit 4) streaming stores, (bit 5) tile order by
    // column bands
    if (c->p.precision == MRTFD_BF16X3) {
        const bool bands = ((c->p.nx + 63) / 64) % 8 == 0;
        for (int r = 1; r <= 2; ++r)
            for (int o = 0; o <= (bands ? 1 : 0); ++o) {
                cands.push_back({MRTFD_KERNEL_MFMA, r | (o << 5)});
                cands.push_back({MRTFD_KERNEL_MFMA, r | 16 | (o << 5)});
            }
    } else if (c->p.kernel == MRTFD_KERNEL_SIMPLE) {
        cands.push_back({MRTFD_KERNEL_SIMPLE, 0});
    } else {
        const bool bands = ((c->p.nx + 63) / 64) % 8 == 0;
        for (int r = 1; r <= (is64(c) ? 1 : 2); ++r) {
            if (c->p.rows && r != c->p.rows) continue;
            for (int o = 0; o <= (bands ? 1 : 0); ++o) {
                cands.push_back({MRTFD_KERNEL_ROWS, r | (o << 5)});
                cands.push_back({MRTFD_KERNEL_ROWS, r | 16 | (o << 5)});
            }
        }
        if (c->p.kernel == MRTFD_KERNEL_AUTO) cands.push_back({MRTFD_KERNEL_SIMPLE, 0});
    }
    c->kernel = cands[0].first;
    c->seg = cands[0].second;
    if (cands.size() == 1) {
        c->tuned = true;
        return MRTFD_OK;
    }
    const double cells = (double)c->p.nx * c->p.ny;
    // at least ~1.5 ms of steps per timed trial (about 3.4e7 node updates),
    // 8 to 32 steps
    const long long reps = 2 * (long long)std::max(4.0, std::min(16.0, 3.4e7 / cells));
    const long long warm = 2;
    const int passes = 2;
    if (avail < passes * (long long)cands.size() * (reps + warm)) return MRTFD_OK;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    std::vector<float> t(cands.size(), 1e30f);
    int rc = MRTFD_OK;
    for (size_t trial = 0; trial < passes * cands.size() && rc == MRTFD_OK; ++trial) {
        const size_t ci = trial % cands.size();
        const std::pair<int, int> cand = cands[ci];
        c->kernel = cand.first;
        c->seg = cand.second;
        hipError_t e = direct_steps(c, warm);
        e = e == hipSuccess ? hipEventRecord(e0, c->stream) : e;
        e = e == hipSuccess ? direct_steps(c, reps) : e;
        e = e == hipSuccess ? hipEventRecord(e1, c->stream) : e;
        e = e == hipSuccess ? hipEventSynchronize(e1) : e;
        float ms = 0.f;
        e = e == hipSuccess ? hipEventElapsedTime(&ms, e0, e1) : e;
        if (e != hipSuccess) {
            rc = set_err(c, MRTFD_ERR_HIP, "autotune: %s", hipGetErrorString(e));
            break;
        }
        *taken += warm + reps;
        t[ci] = std::min(t[ci], ms);
    }
    std::pair<int, int> pick = cands[0];
    float best = t[0];
    for (size_t ci = 1; ci < cands.size(); ++ci)
        if (t[ci] < best) {
            best = t[ci];
            pick = cands[ci];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->kernel = pick.first;
    c->seg = pick.second;
    // graphs captured by earlier, shorter calls hold the default variant:
    // wait until none is in flight (an error may have cut the trials short
    // of their own synchronisation), then drop them; they are rebuilt on the
    // next replay
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (rc == MRTFD_OK) {
        c->tuned = true;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = pick;
    }
    return rc;
}

// The screen's own check of p: positive finite dx, dy, dt and finite,
// non-negative rates; dt s_k above 1 is allowed (finding out what happens
// there is what the screen is for), the grid and boundary fields are not used.
bool screen_params_ok(const mrtfd_params *p, bool rates)
{
    if (!p) return false;
    for (double x : {p->dx, p->dy, p->dt})
        if (!(x > 0.0) || !std::isfinite(x)) return false;
    if (rates)
        for (int k = 0; k < NQ; ++k)
            if (!(p->s[k] >= 0.0) || !std::isfinite(p->s[k])) return false;
    return true;
}

}  // namespace

// ------------------------------------------------------------------- C ABI

extern "C" {

const char *mrtfd_status_string(int32_t s)
{
    switch (s) {
    case MRTFD_OK: return "ok";
    case MRTFD_ERR_ARG: return "invalid argument";
    case MRTFD_ERR_HIP: return "HIP runtime error";
    case MRTFD_ERR_UNSTABLE: return "parameters outside the stable range";
    case MRTFD_ERR_NONFINITE: return "non-finite values in the state";
    case MRTFD_ERR_STATE: return "call out of order";
    case MRTFD_ERR_UNSUPPORTED: return "unsupported mode";
    default: return "unknown status";
    }
}

const char *mrtfd_last_error(const mrtfd_ctx *c) { return c ? c->err : "no context"; }

int32_t mrtfd_model(double *v, double *M, double *Minv)
{
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    if (v) std::memcpy(v, m.v, sizeof m.v);
    if (M) std::memcpy(M, m.M, sizeof m.M);
    if (Minv) std::memcpy(Minv, m.Minv, sizeof m.Minv);
    return MRTFD_OK;
}

int32_t mrtfd_screen(const mrtfd_params *p, const double state[4], const double *d_theta, int32_t n,
                     double *d_eig, double *d_rho, void *stream)
{
    if (!p || !state) return MRTFD_ERR_ARG;
    if (!screen_params_ok(p, true)) return MRTFD_ERR_ARG;
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(state[c])) return MRTFD_ERR_ARG;
    if (!(state[0] > 0) || !(state[3] > 0)) return MRTFD_ERR_ARG;
    if (n < 0) return MRTFD_ERR_ARG;
    if (n == 0) return MRTFD_OK;
    if (!d_theta || (!d_eig && !d_rho)) return MRTFD_ERR_ARG;
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    ScreenCoef S;
    screen_coef(m, *p, state, S);
    return launch_screen(S, d_theta, n, d_eig, d_rho, static_cast<hipStream_t>(stream)) == hipSuccess
               ? MRTFD_OK
               : MRTFD_ERR_HIP;
}

int32_t mrtfd_screen_sets(const mrtfd_params *p, int32_t nsets, const double *d_states, const double *d_rates,
                          const double *d_theta, int32_t n, double *d_rho, double *d_max, void *stream)
{
    if (!screen_params_ok(p, false)) return MRTFD_ERR_ARG;
    if (nsets < 0 || n < 0) return MRTFD_ERR_ARG;
    if ((long long)nsets * n > 0x7fffffffLL) return MRTFD_ERR_ARG;
    if ((long long)nsets * n == 0) return MRTFD_OK;
    if (!d_states || !d_rates || !d_theta || (!d_rho && !d_max)) return MRTFD_ERR_ARG;
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    static double host_model[2 * NQ * NQ + 2 * NQ];
    static std::once_flag once;
    std::call_once(once, [&] {
        std::memcpy(host_model, m.M, sizeof(double) * NQ * NQ);
        std::memcpy(host_model + NQ * NQ, m.Minv, sizeof(double) * NQ * NQ);
        std::memcpy(host_model + 2 * NQ * NQ, m.v, sizeof(double) * 2 * NQ);
    });
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || screen_model_ready(dev, host_model) != hipSuccess) return MRTFD_ERR_HIP;
    ScreenSetArgs a{d_states, d_rates, d_theta, d_rho, d_max, nsets, n, p->dx, p->dy, p->dt};
    return launch_screen_sets(a, static_cast<hipStream_t>(stream)) == hipSuccess ? MRTFD_OK : MRTFD_ERR_HIP;
}

int32_t mrtfd_ref_populations(const mrtfd_params *p, double out[16])
{
    if (!p || !out) return MRTFD_ERR_ARG;
    if (check(p, nullptr, 0) != MRTFD_OK) return MRTFD_ERR_ARG;
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    ref_populations(m, *p, out);
    return MRTFD_OK;
}

int32_t mrtfd_struct_sizes(size_t *params_size, size_t *side_size)
{
    if (params_size) *params_size = sizeof(mrtfd_params);
    if (side_size) *side_size = sizeof(mrtfd_side);
    return MRTFD_OK;
}

int32_t mrtfd_check_params(const mrtfd_params *p, char *msg, size_t msg_len)
{
    try {
        return check(p, msg, msg_len);
    } catch (...) {
        return MRTFD_ERR_ARG;
    }
}

size_t mrtfd_workspace_bytes(const mrtfd_params *p)
{
    try {
        if (check(p, nullptr, 0) != MRTFD_OK) return 0;
        return layout(*p).total;
    } catch (...) {
        return 0;
    }
}

int32_t mrtfd_create(const mrtfd_params *p, void *d_ws, size_t ws_bytes, void *stream,
                     mrtfd_ctx **out)
{
    if (!out) return MRTFD_ERR_ARG;
    *out = nullptr;
    char msg[256];
    int rc = check(p, msg, sizeof msg);
    if (rc != MRTFD_OK) return rc;
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    const Layout L = layout(*p);
    if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return MRTFD_ERR_ARG;
    mrtfd_ctx *c = new (std::nothrow) mrtfd_ctx();
    if (!c) return MRTFD_ERR_ARG;
    c->p = *p;
    c->F = make_field(*p);
    c->L = L;
    c->ws = static_cast<char *>(d_ws);
    if (p->precision == MRTFD_FP64) {
        c->f64[0] = reinterpret_cast<double *>(c->ws + L.fA);
        c->f64[1] = reinterpret_cast<double *>(c->ws + L.fB);
    } else {
        c->f[0] = reinterpret_cast<float *>(c->ws + L.fA);
        c->f[1] = reinterpret_cast<float *>(c->ws + L.fB);
    }
    c->partials = reinterpret_cast<double *>(c->ws + L.partials);
    c->sums = reinterpret_cast<double *>(c->ws + L.sums);
    c->d_step = reinterpret_cast<long long *>(c->ws + L.step);
    c->d_flag = reinterpret_cast<int *>(c->ws + L.flag);
    c->d_bf3 = reinterpret_cast<Bf3Ops *>(c->ws + L.bf3);
    c->flux = reinterpret_cast<double *>(c->ws + L.flux);
    c->outflow = reinterpret_cast<double *>(c->ws + L.outflow);
    for (int q = 0; q < NQ; ++q) {
        const double vx = m.v[q][0], vy = m.v[q][1];
        c->FC.cx[q][0] = p->dt / p->dx * vx / 2.0;
        c->FC.cx[q][1] = p->dt / p->dx * vx * vx * p->dt / (2.0 * p->dx);
        c->FC.cy[q][0] = p->dt / p->dy * vy / 2.0;
        c->FC.cy[q][1] = p->dt / p->dy * vy * vy * p->dt / (2.0 * p->dy);
        for (int k = 0; k < 4; ++k) c->FC.w[k][q] = m.M[k][q];
    }
    c->stream = static_cast<hipStream_t>(stream);
    fill_consts(m, *p, c->K);
    fill_consts(m, *p, c->K64);
    if (!fill_bf3(c->K, c->h_bf3) && p->precision == MRTFD_BF16X3) {
        delete c;  // a weight that its BF16 parts do not hold exactly
        return MRTFD_ERR_UNSUPPORTED;
    }
    ref_populations(m, *p, c->fref);
    // outflow of the uniform f_ref through one node of each side per step
    // (its face value is v f_ref), added to the budget's totals on readout
    for (int s = 0; s < 4; ++s)
        for (int k = 0; k < 4; ++k) {
            double a = 0.0;
            for (int q = 0; q < NQ; ++q) {
                const double c0 = s < 2 ? c->FC.cx[q][0] : c->FC.cy[q][0];
                a += c->FC.w[k][q] * 2.0 * c0 * c->fref[q];
            }
            c->ref_out[s][k] = (s == 0 || s == 2) ? -a : a;
        }
    for (int k = 0; k < 4; ++k)
        for (int q = 0; q < NQ; ++q) c->W.w[k][q] = m.M[k][q];
    {
        // the reference state's share of the sums: its moments (rho0, 0, 0,
        // e0) at every node
        double rho0, T0;
        ref_state(*p, rho0, T0);
        const double nodes = (double)p->nx * (double)p->ny;
        c->W.add[0] = nodes * rho0;
        c->W.add[1] = c->W.add[2] = 0.0;
        c->W.add[3] = nodes * (rho0 * T0);
    }
    fill_ghosts(m, *p, c->fref, c->ws + L.kcopy, c->ws + L.gcopy, c->ws + L.fcopy, c->G);
    fill_ghosts(m, *p, c->fref, c->ws + L.kcopy, c->ws + L.gcopy, c->ws + L.fcopy, c->G64);
    // default until tuned: rows kernel, one row per wave, plain stores
    c->kernel = p->kernel == MRTFD_KERNEL_SIMPLE ? MRTFD_KERNEL_SIMPLE : MRTFD_KERNEL_ROWS;
    c->seg = p->kernel == MRTFD_KERNEL_SIMPLE ? 0 : 1;
    if (p->kernel == MRTFD_KERNEL_ROWS && p->rows) {
        c->seg = p->rows;
        c->tuned = true;
    }
    if (p->precision == MRTFD_BF16X3) {  // stores and tile order autotuned
        c->kernel = MRTFD_KERNEL_MFMA;
        c->seg = 1;
        c->tuned = false;
    }

    hipError_t e = hipGetDevice(&c->device);
    // this device's copy of the library scratch (mrtfd_sums_noalloc)
    if (e == hipSuccess) e = scratch_address(c->device, &c->scratch);
    if (e == hipSuccess && p->flux_budget) {
        e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = launch_zero(c->ws, L.total, c->stream);
    if (e == hipSuccess && poison_padding())  // both copies of f: a quiet NaN everywhere
        e = launch_fill(c->ws + L.fA, L.partials - L.fA, 0x7FC00000u, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_bf3, &c->h_bf3, sizeof(Bf3Ops), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = p->precision == MRTFD_FP64
                ? hipMemcpyAsync(c->ws + L.kcopy, &c->K64, sizeof(Consts64), hipMemcpyHostToDevice, c->stream)
                : hipMemcpyAsync(c->ws + L.kcopy, &c->K, sizeof(Consts), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = p->precision == MRTFD_FP64
                ? hipMemcpyAsync(c->ws + L.gcopy, &c->G64, sizeof(Ghosts64), hipMemcpyHostToDevice, c->stream)
                : hipMemcpyAsync(c->ws + L.gcopy, &c->G, sizeof(Ghosts), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->ws + L.fcopy, &c->FC, sizeof(FluxCoef), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        release(c);
        return MRTFD_ERR_HIP;
    }
    *out = c;
    return MRTFD_OK;
}

int32_t mrtfd_destroy(mrtfd_ctx *c)
{
    if (!c) return MRTFD_ERR_ARG;
    release(c);
    return MRTFD_OK;
}

int32_t mrtfd_init_macro(mrtfd_ctx *c, const float *rho, const float *ux, const float *uy,
                         const float *T)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!rho || !ux || !uy || !T) return set_err(c, MRTFD_ERR_ARG, "init_macro: NULL field");
    HIPCHK(c, launch_zero(c->d_flag, sizeof(int), c->stream));
    c->cur = 0;
    if (is64(c))
        HIPCHK(c, launch_init(c->F, c->K64, c->f64[0], rho, ux, uy, T, c->d_flag, c->stream));
    else
        HIPCHK(c, launch_init(c->F, c->K, c->f[0], rho, ux, uy, T, c->d_flag, c->stream));
    HIPCHK(c, launch_counter_set(c->d_step, 0, c->stream));
    if (c->p.flux_budget)
        HIPCHK(c, launch_zero(c->flux, c->L.outflow - c->L.flux, c->stream));
    c->budget_steps = 0;
    c->step = 0;
    c->initialised = true;
    return MRTFD_OK;
}

int32_t mrtfd_set_f(mrtfd_ctx *c, const float *src)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!src) return set_err(c, MRTFD_ERR_ARG, "set_f: NULL array");
    if (is64(c))
        HIPCHK(c, launch_unpack(c->F, src, c->f64[c->cur], c->stream));
    else
        HIPCHK(c, launch_unpack(c->F, src, c->f[c->cur], c->stream));
    if (c->p.flux_budget)
        HIPCHK(c, launch_zero(c->flux, c->L.outflow - c->L.flux, c->stream));
    c->budget_steps = 0;
    c->initialised = true;
    return MRTFD_OK;
}

int32_t mrtfd_get_f(mrtfd_ctx *c, float *dst)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!dst) return set_err(c, MRTFD_ERR_ARG, "get_f: NULL array");
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "get_f before init");
    if (is64(c))
        HIPCHK(c, launch_pack(c->F, c->f64[c->cur], dst, c->stream));
    else
        HIPCHK(c, launch_pack(c->F, c->f[c->cur], dst, c->stream));
    return MRTFD_OK;
}

int32_t mrtfd_set_f64(mrtfd_ctx *c, const double *src)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!src) return set_err(c, MRTFD_ERR_ARG, "set_f64: NULL array");
    if (is64(c))
        HIPCHK(c, launch_unpack(c->F, src, c->f64[c->cur], c->stream));
    else
        HIPCHK(c, launch_unpack(c->F, src, c->f[c->cur], c->stream));
    if (c->p.flux_budget)
        HIPCHK(c, launch_zero(c->flux, c->L.outflow - c->L.flux, c->stream));
    c->budget_steps = 0;
    c->initialised = true;
    return MRTFD_OK;
}

int32_t mrtfd_get_f64(mrtfd_ctx *c, double *dst)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!dst) return set_err(c, MRTFD_ERR_ARG, "get_f64: NULL array");
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "get_f64 before init");
    if (is64(c))
        HIPCHK(c, launch_pack(c->F, c->f64[c->cur], dst, c->stream));
    else
        HIPCHK(c, launch_pack(c->F, c->f[c->cur], dst, c->stream));
    return MRTFD_OK;
}

int32_t mrtfd_step(mrtfd_ctx *c, int64_t nsteps)
{
    if (!c) return MRTFD_ERR_ARG;
    if (nsteps < 0) return set_err(c, MRTFD_ERR_ARG, "nsteps must be >= 0");
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "step before init");
    if (nsteps == 0) return MRTFD_OK;
    c->budget_steps += nsteps;
    long long left = nsteps;
    if (!c->tuned) {
        long long taken = 0;
        int rc = autotune(c, left, &taken);
        if (rc != MRTFD_OK) return rc;
        left -= taken;
    }
    const int G = c->p.graph_steps;
    if (G > 0) {
        while (left >= G) {
            if (!c->graph[c->cur]) {
                int rc = build_graph(c, c->cur);
                if (rc != MRTFD_OK) return rc;
            }
            HIPCHK(c, hipGraphLaunch(c->graph[c->cur], c->stream));
            left -= G;  // G is even: the state ends in the copy it started from
            c->step += G;
        }
    }
    HIPCHK(c, direct_steps(c, left));
    return MRTFD_OK;
}

int32_t mrtfd_read_macro(mrtfd_ctx *c, float *rho, float *ux, float *uy, float *T, float *p)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "read_macro before init");
    if (is64(c))
        HIPCHK(c, launch_read_macro(c->F, c->K64, c->f64[c->cur], rho, ux, uy, T, p, c->stream));
    else
        HIPCHK(c, launch_read_macro(c->F, c->K, c->f[c->cur], rho, ux, uy, T, p, c->stream));
    return MRTFD_OK;
}

int32_t mrtfd_sums(mrtfd_ctx *c, double out[4])
{
    if (!c || !out) return MRTFD_ERR_ARG;
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "sums before init");
    if (is64(c))
        HIPCHK(c, launch_sums(c->F, c->W, c->f64[c->cur], c->partials, c->sums, c->stream));
    else
        HIPCHK(c, launch_sums(c->F, c->W, c->f[c->cur], c->partials, c->sums, c->stream));
    double h[4];
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(h, c->sums, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&flag, c->d_flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < 4; ++k) out[k] = h[k];
    if (flag) return set_err(c, MRTFD_ERR_ARG, "initial state had rho <= 0, T <= 0 or non-finite values");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(h[k])) return set_err(c, MRTFD_ERR_NONFINITE, "sum %d is not finite", k);
    return MRTFD_OK;
}

int32_t mrtfd_sums_noalloc(mrtfd_ctx *c, double *d_out)
{
    if (!c) return MRTFD_ERR_ARG;
    if (!d_out) return set_err(c, MRTFD_ERR_ARG, "sums_noalloc: NULL output");
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "sums_noalloc before init");
    if (!c->scratch) return set_err(c, MRTFD_ERR_STATE, "sums_noalloc: no library scratch");
    const int nb = sums_blocks(c->F);
    if (4 * nb > SCRATCH_DOUBLES)
        return set_err(c, MRTFD_ERR_ARG, "sums_noalloc: %d partial sums exceed the scratch of %d",
                       4 * nb, SCRATCH_DOUBLES);
    if (is64(c))
        HIPCHK(c, launch_sums(c->F, c->W, c->f64[c->cur], c->scratch, d_out, c->stream));
    else
        HIPCHK(c, launch_sums(c->F, c->W, c->f[c->cur], c->scratch, d_out, c->stream));
    return MRTFD_OK;
}

int32_t mrtfd_outflow(mrtfd_ctx *c, double out[16])
{
    if (!c || !out) return MRTFD_ERR_ARG;
    if (!c->p.flux_budget) return set_err(c, MRTFD_ERR_STATE, "outflow needs flux_budget = 1 at create");
    if (!c->initialised) return set_err(c, MRTFD_ERR_STATE, "outflow before init");
    HIPCHK(c, launch_flux_totals(c->p.nx, c->p.ny, c->flux, c->outflow, c->stream));
    double h[16];
    HIPCHK(c, hipMemcpyAsync(h, c->outflow, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the kernels take face values of the stored g = f - f_ref; the uniform
    // f_ref adds the same outflow through every side node in every step
    for (int sd = 0; sd < 4; ++sd) {
        const double len = sd < 2 ? (double)c->p.ny : (double)c->p.nx;
        for (int k = 0; k < 4; ++k) h[4 * sd + k] += (double)c->budget_steps * len * c->ref_out[sd][k];
    }
    for (int k = 0; k < 16; ++k) out[k] = h[k];
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(h[k])) return set_err(c, MRTFD_ERR_NONFINITE, "outflow %d is not finite", k);
    return MRTFD_OK;
}

int32_t mrtfd_time(mrtfd_ctx *c, int64_t *step, double *t)
{
    if (!c) return MRTFD_ERR_ARG;
    if (step) *step = c->step;
    if (t) *t = (double)c->step * c->p.dt;
    return MRTFD_OK;
}

int32_t mrtfd_set_step(mrtfd_ctx *c, int64_t step)
{
    if (!c) return MRTFD_ERR_ARG;
    if (step < 0) return set_err(c, MRTFD_ERR_ARG, "step must be >= 0");
    HIPCHK(c, launch_counter_set(c->d_step, step, c->stream));
    c->step = step;
    return MRTFD_OK;
}

int32_t mrtfd_kernel_info(mrtfd_ctx *c, int32_t *kernel, int32_t *rows, int32_t *streaming,
                          int32_t *tile_order)
{
    if (!c) return MRTFD_ERR_ARG;
    if (kernel) *kernel = c->kernel;
    if (rows) *rows = c->seg & 15;
    if (streaming) *streaming = (c->seg >> 4) & 1;
    if (tile_order) *tile_order = (c->seg >> 5) & 1;
    return MRTFD_OK;
}

}  // extern "C"

// ------------------------------------------------------------ tube batches

namespace {

struct BatchLayout {
    size_t fA, fB, tubes, states, items, kcopy, total;
    long long ncols;
    size_t max_items;
};

const int kTubeSegs[] = {32, 48, 56};

int batch_check(const mrtfd_batch_params *p, const int32_t *n, char *msg, size_t len)
{
    auto fail = [&](int code, const char *fmt, ...) {
        if (msg && len) {
            va_list ap;
            va_start(ap, fmt);
            std::vsnprintf(msg, len, fmt, ap);
            va_end(ap);
        }
        return code;
    };
    if (!p || !n) return fail(MRTFD_ERR_ARG, "NULL argument");
    if (p->ntubes < 1) return fail(MRTFD_ERR_ARG, "ntubes must be >= 1");
    if (!(p->dx > 0) || !(p->dt > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dt))
        return fail(MRTFD_ERR_ARG, "dx and dt must be positive and finite");
    for (int k = 4; k < NQ; ++k) {
        if (!(p->s[k] >= 0) || !std::isfinite(p->s[k])) return fail(MRTFD_ERR_ARG, "bad s_%d", k + 1);
        if (p->dt * p->s[k] > 1.0 + 1e-12)
            return fail(MRTFD_ERR_UNSTABLE, "dt * s_%d = %g exceeds 1", k + 1, p->dt * p->s[k]);
    }
    if (6.0 * p->dt / p->dx > 1.0) return fail(MRTFD_ERR_UNSTABLE, "Courant number 6 dt / dx exceeds 1");
    if (p->seg_cols && p->round_steps && !tubes_config_built(p->seg_cols, p->round_steps))
        return fail(MRTFD_ERR_ARG, "seg_cols/round_steps pair not built");
    if (p->seg_cols && p->seg_cols != 32 && p->seg_cols != 48 && p->seg_cols != 56)
        return fail(MRTFD_ERR_ARG, "seg_cols must be 0, 32, 48 or 56");
    if (p->round_steps && p->round_steps != 4 && p->round_steps != 8 && p->round_steps != 16)
        return fail(MRTFD_ERR_ARG, "round_steps must be 0, 4, 8 or 16");
    long long total = 0;
    for (int k = 0; k < p->ntubes; ++k) {
        if (n[k] < 3) return fail(MRTFD_ERR_ARG, "tube %d has %d < 3 columns", k, n[k]);
        total += n[k];
    }
    if (4LL * NQ * TUBE_ROWS * total >= (1LL << 34)) return fail(MRTFD_ERR_ARG, "batch too large");
    if (msg && len) msg[0] = 0;
    return MRTFD_OK;
}

BatchLayout batch_layout(const mrtfd_batch_params *p, const int32_t *n)
{
    BatchLayout L;
    L.ncols = 0;
    L.max_items = 0;
    for (int k = 0; k < p->ntubes; ++k) {
        L.ncols += n[k];
        L.max_items += (size_t)((n[k] + 31) / 32);
    }
    const size_t fbytes = align256((size_t)NQ * TUBE_ROWS * (size_t)L.ncols * sizeof(float));
    L.fA = 0;
    L.fB = fbytes;
    L.tubes = 2 * fbytes;
    L.states = L.tubes + align256((size_t)p->ntubes * sizeof(TubeInfo));
    L.items = L.states + align256((size_t)p->ntubes * 8 * sizeof(float));
    L.kcopy = L.items + align256(L.max_items * sizeof(TubeItem));
    L.total = L.kcopy + align256(sizeof(Consts));
    return L;
}

}  // namespace

struct mrtfd_batch {
    mrtfd_batch_params p;
    BatchLayout L;
    TubeGrid TG;
    Consts K;
    std::vector<int> n, start, order;
    std::vector<long long> steps;
    std::vector<TubeInfo> info;
    std::vector<float> states;
    std::vector<TubeItem> items;      // for the chosen seg, tubes by decreasing steps
    std::vector<int> round_items;     // items active in each round
    std::vector<int> final_copy;      // copy holding each tube's state
    char *ws = nullptr;
    float *f[2] = {nullptr, nullptr};
    TubeInfo *d_tubes = nullptr;
    float *d_states = nullptr;
    TubeItem *d_items = nullptr;
    const Consts *d_k = nullptr;  // device copy of K, read by the tube kernel
    hipStream_t stream = nullptr, cap = nullptr;
    hipGraphExec_t graph = nullptr;
    int seg = 0, ks = 0, max_n = 0;
    bool initialised = false, done = false;
    char err[512] = {0};
};

namespace {

int bset_err(mrtfd_batch *b, int code, const char *fmt, ...)
{
    if (b) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(b->err, sizeof b->err, fmt, ap);
        va_end(ap);
    }
    return code;
}

#define BHIPCHK(b, expr)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bset_err(b, MRTFD_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// Items of all tubes (in order of decreasing step count) for a work-item
// width; round_items[r] = number of leading items whose tube still runs in
// round r.
void build_items(mrtfd_batch *b, int seg, int ks, std::vector<TubeItem> &items,
                 std::vector<int> &round_items)
{
    items.clear();
    std::vector<size_t> first(b->order.size() + 1, 0);
    for (size_t r = 0; r < b->order.size(); ++r) {
        const int k = b->order[r];
        first[r] = items.size();
        for (int x0 = 0; x0 < b->n[k]; x0 += seg) items.push_back(TubeItem{k, x0});
    }
    first[b->order.size()] = items.size();
    long long max_steps = b->order.empty() ? 0 : b->steps[b->order[0]];
    const long long rounds = (max_steps + ks - 1) / ks;
    round_items.assign((size_t)rounds, 0);
    size_t t = b->order.size();  // tubes still running: a prefix of the order
    for (long long r = 0; r < rounds; ++r) {
        while (t > 0 && b->steps[b->order[t - 1]] <= r * ks) --t;
        round_items[(size_t)r] = (int)first[t];
    }
}

hipError_t enqueue_rounds(mrtfd_batch *b, hipStream_t s)
{
    const int R = (int)b->round_items.size();
    for (int r = 0; r < R; ++r) {
        hipError_t e = launch_tubes(b->TG, b->d_k, b->d_tubes, b->d_items, b->round_items[r], r,
                                    b->seg, b->ks, b->f[r & 1], b->f[(r + 1) & 1], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Pick the work-item width and steps per round (all give the same bits) by
// timing each candidate on two rounds of the batch itself: round 0, where
// every tube runs, and the round a quarter of the way through the longest
// run, where the short tubes are done.  Each trial launch reads copy 0 and
// writes copy 1, which the real run overwrites.  Two passes over the
// candidates, each keeping its faster pass (the first launches of a new
// shape run slower).
int batch_autotune(mrtfd_batch *b)
{
    if (b->seg && b->ks) return MRTFD_OK;
    static std::mutex mu;
    static std::map<std::vector<int>, std::pair<int, int>> cache;
    std::vector<int> key(b->n);
    for (long long v : b->steps) key.push_back((int)std::min<long long>(v, 1 << 30));
    key.push_back(b->p.seg_cols);
    key.push_back(b->p.round_steps);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            b->seg = it->second.first;
            b->ks = it->second.second;
            return MRTFD_OK;
        }
    }
    struct Cand {
        int seg, ks;
        std::vector<TubeItem> items;
        std::vector<int> ri;
        double work[2];
        int round[2];
    };
    std::vector<Cand> cands;
    for (int seg : kTubeSegs) {
        if (b->p.seg_cols && seg != b->p.seg_cols) continue;
        for (int ks : {4, 8, 16}) {
            if (b->p.round_steps && ks != b->p.round_steps) continue;
            if (!tubes_config_built(seg, ks)) continue;
            Cand c;
            c.seg = seg;
            c.ks = ks;
            build_items(b, seg, ks, c.items, c.ri);
            if (c.ri.empty() || c.ri[0] == 0) continue;
            const int R = (int)c.ri.size();
            c.round[0] = 0;
            c.round[1] = R / 4;
            for (int t = 0; t < 2; ++t) {  // node updates of the trial round
                double w = 0.0;
                const long long r = c.round[t];
                for (int k = 0; k < b->p.ntubes; ++k) {
                    const long long left = b->steps[k] - r * ks;
                    if (left > 0) w += (double)b->n[k] * TUBE_ROWS * (double)std::min<long long>(ks, left);
                }
                c.work[t] = w;
            }
            cands.push_back(std::move(c));
        }
    }
    if (cands.empty()) return bset_err(b, MRTFD_ERR_ARG, "batch autotune: no candidate");
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    int rc = MRTFD_OK;
    std::vector<double> rate(cands.size(), 0.0);
    for (int pass = 0; pass < 2 && rc == MRTFD_OK; ++pass) {
        for (size_t ci = 0; ci < cands.size() && rc == MRTFD_OK; ++ci) {
            Cand &c = cands[ci];
            hipError_t e = hipMemcpyAsync(b->d_items, c.items.data(), c.items.size() * sizeof(TubeItem),
                                          hipMemcpyHostToDevice, b->stream);
            double work = 0.0;
            float total = 0.f;
            for (int t = 0; t < 2 && e == hipSuccess; ++t) {
                const int r = c.round[t], ni = c.ri[(size_t)r];
                if (ni == 0) continue;
                // one launch to warm the shape, then two timed
                e = launch_tubes(b->TG, b->d_k, b->d_tubes, b->d_items, ni, r, c.seg, c.ks, b->f[0],
                                 b->f[1], b->stream);
                if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
                for (int rep = 0; rep < 2 && e == hipSuccess; ++rep)
                    e = launch_tubes(b->TG, b->d_k, b->d_tubes, b->d_items, ni, r, c.seg, c.ks, b->f[0],
                                     b->f[1], b->stream);
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                total += ms;
                work += 2.0 * c.work[t];
            }
            if (e != hipSuccess) {
                rc = bset_err(b, MRTFD_ERR_HIP, "batch autotune: %s", hipGetErrorString(e));
                break;
            }
            rate[ci] = std::max(rate[ci], work / std::max(1e-6, (double)total));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    size_t pick = 0;
    for (size_t ci = 1; ci < cands.size(); ++ci)
        if (rate[ci] > rate[pick]) pick = ci;
    b->seg = cands[pick].seg;
    b->ks = cands[pick].ks;
    if (rc == MRTFD_OK) {
        std::lock_guard<std::mutex> lk(mu);
        cache[key] = std::make_pair(b->seg, b->ks);
    }
    return rc;
}

}  // namespace

extern "C" {

size_t mrtfd_batch_workspace_bytes(const mrtfd_batch_params *p, const int32_t *n)
{
    try {
        if (batch_check(p, n, nullptr, 0) != MRTFD_OK) return 0;
        return batch_layout(p, n).total;
    } catch (...) {
        return 0;
    }
}

int32_t mrtfd_batch_create(const mrtfd_batch_params *p, const int32_t *n, const int64_t *steps,
                           const double *left, const double *right, void *d_ws, size_t ws_bytes,
                           void *stream, mrtfd_batch **out)
{
    if (!out) return MRTFD_ERR_ARG;
    *out = nullptr;
    int rc = batch_check(p, n, nullptr, 0);
    if (rc != MRTFD_OK) return rc;
    if (!steps || !left || !right) return MRTFD_ERR_ARG;
    for (int k = 0; k < p->ntubes; ++k) {
        if (steps[k] < 0) return MRTFD_ERR_ARG;
        for (const double *st : {left + 4 * k, right + 4 * k}) {
            if (!(st[0] > 0) || !(st[3] > 0)) return MRTFD_ERR_ARG;
            for (int c = 0; c < 4; ++c)
                if (!std::isfinite(st[c])) return MRTFD_ERR_ARG;
        }
    }
    const Model &m = model();
    if (!m.ok) return MRTFD_ERR_ARG;
    const BatchLayout L = batch_layout(p, n);
    if (!d_ws || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return MRTFD_ERR_ARG;
    mrtfd_batch *b = new (std::nothrow) mrtfd_batch();
    if (!b) return MRTFD_ERR_ARG;
    try {
        b->p = *p;
        b->L = L;
        b->ws = static_cast<char *>(d_ws);
        b->f[0] = reinterpret_cast<float *>(b->ws + L.fA);
        b->f[1] = reinterpret_cast<float *>(b->ws + L.fB);
        b->d_tubes = reinterpret_cast<TubeInfo *>(b->ws + L.tubes);
        b->d_states = reinterpret_cast<float *>(b->ws + L.states);
        b->d_items = reinterpret_cast<TubeItem *>(b->ws + L.items);
        b->d_k = reinterpret_cast<const Consts *>(b->ws + L.kcopy);
        b->stream = static_cast<hipStream_t>(stream);
        b->TG.ncols = (int)L.ncols;
        b->TG.plane = (long long)TUBE_ROWS * L.ncols;
        // the step constants: same construction as a single grid with dx = dy
        mrtfd_params gp;
        std::memset(&gp, 0, sizeof gp);
        gp.dx = gp.dy = p->dx;
        gp.dt = p->dt;
        for (int k = 0; k < NQ; ++k) gp.s[k] = p->s[k];
        fill_consts(m, gp, b->K);
        b->n.assign(n, n + p->ntubes);
        b->steps.assign(steps, steps + p->ntubes);
        b->start.resize(p->ntubes);
        b->info.resize(p->ntubes);
        b->states.resize((size_t)p->ntubes * 8);
        long long acc = 0;
        for (int k = 0; k < p->ntubes; ++k) {
            b->start[k] = (int)acc;
            acc += n[k];
            b->max_n = std::max(b->max_n, n[k]);
            TubeInfo &t = b->info[k];
            std::memset(&t, 0, sizeof t);
            t.n = n[k];
            t.start = b->start[k];
            t.steps = (int)std::min<long long>(steps[k], (long long)1 << 30);
            double fe[NQ];
            feq_host(m, left[4 * k], left[4 * k + 1], left[4 * k + 2], left[4 * k + 3], fe);
            for (int q = 0; q < NQ; ++q) t.feq_left[q] = (float)fe[q];
            feq_host(m, right[4 * k], right[4 * k + 1], right[4 * k + 2], right[4 * k + 3], fe);
            for (int q = 0; q < NQ; ++q) t.feq_right[q] = (float)fe[q];
            for (int c = 0; c < 4; ++c) {
                b->states[8 * k + c] = (float)left[4 * k + c];
                b->states[8 * k + 4 + c] = (float)right[4 * k + c];
            }
        }
        b->order.resize(p->ntubes);
        for (int k = 0; k < p->ntubes; ++k) b->order[k] = k;
        std::stable_sort(b->order.begin(), b->order.end(),
                         [&](int a, int c) { return b->steps[a] > b->steps[c]; });
        b->final_copy.assign(p->ntubes, 0);
        if (p->seg_cols && p->round_steps) {
            b->seg = p->seg_cols;
            b->ks = p->round_steps;
        }
    } catch (...) {
        delete b;
        return MRTFD_ERR_ARG;
    }
    hipError_t e = launch_zero(b->ws, L.total, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_tubes, b->info.data(), b->info.size() * sizeof(TubeInfo),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_states, b->states.data(), b->states.size() * sizeof(float),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->ws + L.kcopy, &b->K, sizeof(Consts), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return MRTFD_ERR_HIP;
    }
    *out = b;
    return MRTFD_OK;
}

int32_t mrtfd_batch_init(mrtfd_batch *b)
{
    if (!b) return MRTFD_ERR_ARG;
    BHIPCHK(b, launch_tubes_init(b->TG, b->K, b->d_tubes, b->d_states, b->p.ntubes, b->max_n, b->f[0],
                                 b->stream));
    std::fill(b->final_copy.begin(), b->final_copy.end(), 0);
    b->initialised = true;
    b->done = false;
    return MRTFD_OK;
}

int32_t mrtfd_batch_run(mrtfd_batch *b)
{
    if (!b) return MRTFD_ERR_ARG;
    if (!b->initialised || b->done) return bset_err(b, MRTFD_ERR_STATE, "run needs a fresh mrtfd_batch_init");
    if (!b->seg) {
        int rc = batch_autotune(b);
        if (rc != MRTFD_OK) return rc;
    }
    if (b->items.empty()) {
        build_items(b, b->seg, b->ks, b->items, b->round_items);
        BHIPCHK(b, hipMemcpyAsync(b->d_items, b->items.data(), b->items.size() * sizeof(TubeItem),
                                  hipMemcpyHostToDevice, b->stream));
    }
    if (b->p.use_graph) {
        if (!b->graph) {
            if (!b->cap) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            hipGraph_t g = nullptr;
            BHIPCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_rounds(b, b->cap);
            hipError_t e2 = hipStreamEndCapture(b->cap, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return bset_err(b, MRTFD_ERR_HIP, "batch graph capture failed");
            }
            e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return bset_err(b, MRTFD_ERR_HIP, "batch graph instantiate failed");
        }
        BHIPCHK(b, hipGraphLaunch(b->graph, b->stream));
    } else {
        BHIPCHK(b, enqueue_rounds(b, b->stream));
    }
    for (int k = 0; k < b->p.ntubes; ++k) {
        const long long rounds = (b->steps[k] + b->ks - 1) / b->ks;
        b->final_copy[k] = (int)(rounds & 1);
    }
    b->done = true;
    return MRTFD_OK;
}

int32_t mrtfd_batch_read_macro(mrtfd_batch *b, int32_t tube, float *rho, float *ux, float *uy,
                               float *T, float *pr)
{
    if (!b) return MRTFD_ERR_ARG;
    if (tube < 0 || tube >= b->p.ntubes) return bset_err(b, MRTFD_ERR_ARG, "bad tube index %d", tube);
    if (!b->initialised) return bset_err(b, MRTFD_ERR_STATE, "read before init");
    BHIPCHK(b, launch_tube_macro(b->TG, b->K, b->d_tubes, tube, b->n[tube], b->f[b->final_copy[tube]], rho,
                                 ux, uy, T, pr, b->stream));
    return MRTFD_OK;
}

int32_t mrtfd_batch_get_f(mrtfd_batch *b, int32_t tube, float *dst)
{
    if (!b || !dst) return MRTFD_ERR_ARG;
    if (tube < 0 || tube >= b->p.ntubes) return bset_err(b, MRTFD_ERR_ARG, "bad tube index %d", tube);
    if (!b->initialised) return bset_err(b, MRTFD_ERR_STATE, "read before init");
    BHIPCHK(b, launch_tube_pack(b->TG, b->d_tubes, tube, b->n[tube], b->f[b->final_copy[tube]], dst,
                                b->stream));
    return MRTFD_OK;
}

int32_t mrtfd_batch_info(mrtfd_batch *b, int32_t *seg, int32_t *ks, int32_t *rounds)
{
    if (!b) return MRTFD_ERR_ARG;
    if (seg) *seg = b->seg;
    if (ks) *ks = b->ks;
    if (rounds) *rounds = (int32_t)b->round_items.size();
    return MRTFD_OK;
}

int32_t mrtfd_batch_destroy(mrtfd_batch *b)
{
    if (!b) return MRTFD_ERR_ARG;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return MRTFD_OK;
}

const char *mrtfd_batch_last_error(const mrtfd_batch *b) { return b ? b->err : "no batch"; }

}  // extern "C"
