// HIP kernels (gfx950) of the MRT finite-difference lattice Boltzmann step.
//
// Per interior node and time step (Sect. II-III, appendix):
//   f-hat = M f; equilibria of the nonconserved moments (Eq. 14);
//   dt*C = M^-1 (dt S-hat)(f-hat - f-hat^eq) (Eq. 3);
//   f_new = f - dt [Lax-Wendroff difference of v.grad f] - dt*C (Eq. A.1a-b),
// collision and stencil both on the old state.  FP32 throughout; FP64 only in
// the conservation sums and in the time comparison that picks a boundary
// rule.  The state is stored as g = f - f_ref, f_ref the equilibrium of a
// reference state at rest (zero when none is set): the difference stencil
// is linear and f_ref uniform, so it acts on g unchanged, and the collision
// needs only the reference's conserved moments added back and its one
// nonzero nonconserved equilibrium (f-hat_11) taken out, so that FP32
// rounding scales with |f - f_ref| instead of |f|.  All code is compiled with FMA contraction off: every fused
// multiply-add below is written out, so every kernel variant rounds a node's
// update identically and their results agree bit for bit.
#include <map>
#include <mutex>
#include <type_traits>

#include "mrtfd_internal.h"

namespace mrtfd {
namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------- transforms

// Stage 1 of f-hat = M f for one velocity group (see Consts).
template <bool AXIS, class Real>
__device__ __forceinline__ void group_fwd(Real q0, Real q1, Real q2, Real q3, Real &A,
                                          Real &X, Real &Y, Real &Q)
{
    const Real s02 = q0 + q2, d02 = q0 - q2, s13 = q1 + q3, d13 = q1 - q3;
    A = s02 + s13;
    Q = s02 - s13;
    if (AXIS) {  // (+,0),(0,+),(-,0),(0,-)
        X = d02;
        Y = d13;
    } else {     // (+,+),(-,+),(-,-),(+,-)
        X = d02 - d13;
        Y = d02 + d13;
    }
}

// Inverse butterfly of one group (scales already folded into A, X, Y, Q).
template <bool AXIS, class Real>
__device__ __forceinline__ void group_inv(Real A, Real X, Real Y, Real Q, Real &q0, Real &q1,
                                          Real &q2, Real &q3)
{
    const Real p = A + Q, m = A - Q;
    if (AXIS) {
        q0 = p + X;
        q2 = p - X;
        q1 = m + Y;
        q3 = m - Y;
    } else {
        const Real xy = X + Y, yx = Y - X;
        q0 = p + xy;
        q2 = p - xy;
        q1 = m + yx;
        q3 = m - yx;
    }
}

template <class Real>
__device__ __forceinline__ Real dot4(const Real (&w)[4], const Real (&v)[4])
{
    return fma_(w[3], v[3], fma_(w[2], v[2], fma_(w[1], v[1], w[0] * v[0])));
}

template <class Real>
__device__ __forceinline__ void butterflies(const Real (&f)[NQ], Real (&A)[4], Real (&X)[4],
                                            Real (&Y)[4], Real (&Q)[4])
{
    group_fwd<true>(f[0], f[1], f[2], f[3], A[0], X[0], Y[0], Q[0]);
    group_fwd<true>(f[4], f[5], f[6], f[7], A[1], X[1], Y[1], Q[1]);
    group_fwd<false>(f[8], f[9], f[10], f[11], A[2], X[2], Y[2], Q[2]);
    group_fwd<false>(f[12], f[13], f[14], f[15], A[3], X[3], Y[3], Q[3]);
}

// All 16 moments, m[k] = f-hat_{k+1}.
template <class Real>
__device__ __forceinline__ void moments(const ConstsT<Real> &K, const Real (&f)[NQ], Real (&m)[NQ])
{
    Real A[4], X[4], Y[4], Q[4];
    butterflies(f, A, X, Y, Q);
    m[0] = dot4(K.f0[0], A);
    m[3] = dot4(K.f0[1], A);
    m[10] = dot4(K.f0[2], A);
    m[11] = dot4(K.f0[3], A);
    m[1] = dot4(K.fx[0], X);
    m[6] = dot4(K.fx[1], X);
    m[8] = dot4(K.fx[2], X);
    m[14] = dot4(K.fx[3], X);
    m[2] = dot4(K.fy[0], Y);
    m[7] = dot4(K.fy[1], Y);
    m[9] = dot4(K.fy[2], Y);
    m[15] = dot4(K.fy[3], Y);
    m[4] = fma_(K.fqa[0][1], Q[1], K.fqa[0][0] * Q[0]);
    m[12] = fma_(K.fqa[1][1], Q[1], K.fqa[1][0] * Q[0]);
    m[5] = fma_(K.fqd[0][1], Q[3], K.fqd[0][0] * Q[2]);
    m[13] = fma_(K.fqd[1][1], Q[3], K.fqd[1][0] * Q[2]);
}

// Conserved moments of the stored populations.  The library stores g = f -
// f_ref, f_ref = f^eq of a reference state at rest (rho0, 0, 0, T0) (all
// zero when no reference is set, so that g = f): the moments of g are rho -
// rho0, j_x, j_y, e - e0 with e0 = rho0 T0.
template <class Real>
__device__ __forceinline__ void conserved(const ConstsT<Real> &K, const Real (&f)[NQ], Real &dr,
                                          Real &jx, Real &jy, Real &de)
{
    Real A[4], X[4], Y[4], Q[4];
    butterflies(f, A, X, Y, Q);
    dr = dot4(K.f0[0], A);
    de = dot4(K.f0[1], A);
    jx = dot4(K.fx[0], X);
    jy = dot4(K.fy[0], Y);
}

// Equilibria of the nonconserved moments, Eq. (14a)-(14i), written with
// u = j / rho; moments 12, 15, 16 have zero equilibrium.  P = e - |j|^2/(2 rho).
// Inputs are deviations from the reference state (dr = rho - rho0, de = e -
// e0) and the outputs are the equilibria less the reference's: at rest only
// f-hat_11^eq = 2 e^2 / rho - |j|^4 / (4 rho^3) is nonzero, 2 rho0 T0^2, and
// 2 e^2/rho - 2 e0^2/rho0 = (2/rho) (de (2 e0 + de) - T0 e0 dr) is formed from
// the deviations so that its rounding scales with them.
template <class Real>
struct EqT {
    Real e5, e6, e7, e8, e9, e10, e11, e13, e14;
};

template <class Real>
__device__ __forceinline__ EqT<Real> equilibria(const ConstsT<Real> &K, Real dr, Real jx, Real jy, Real de)
{
    EqT<Real> q;
    const Real rho = K.rho0 + dr, e = K.e0 + de;
    const Real r = Real(1.0) / rho;  // IEEE division
    const Real ux = jx * r, uy = jy * r;
    const Real jux = jx * ux, juy = jy * uy;
    const Real P = fma_(-Real(0.5), jux + juy, e);
    const Real h = e + P;
    const Real uxx = ux * ux, uyy = uy * uy;
    const Real u2 = uxx + uyy;
    q.e5 = jux - juy;                                 // (jx^2 - jy^2) / rho
    q.e6 = jx * uy;                                   // jx jy / rho
    q.e7 = h * ux;                                    // (e + P) jx / rho
    q.e8 = h * uy;                                    // (e + P) jy / rho
    q.e9 = fma_(-Real(3.0), uyy, uxx) * jx;                // (jx^2 - 3 jy^2) jx / rho^2
    q.e10 = fma_(Real(3.0), uxx, -uyy) * jy;               // (3 jx^2 - jy^2) jy / rho^2
    const Real dd = fma_(de, Real(2.0) * K.e0 + de, -(K.Te0 * dr));
    q.e11 = fma_(Real(2.0) * dd, r, (-Real(0.25) * rho) * (u2 * u2));  // 2 e^2/rho - |j|^4/(4 rho^3) - 2 e0^2/rho0
    const Real er = e * r;
    const Real kap = fma_(Real(6.0), er, -Real(2.0) * u2);    // (6 rho e - 2 |j|^2) / rho^2
    q.e13 = kap * q.e5;
    q.e14 = kap * q.e6;
    return q;
}

// dC = dt * C of Eq. (3) for one node.  A single relaxation time (Sect. II,
// S = I / tau) is the case of equal rates: the same arithmetic, so that
// mass, momentum and energy stay exactly out of the back-map.
template <class Real>
__device__ __forceinline__ void collide(const ConstsT<Real> &K, const Real (&f)[NQ], Real (&dC)[NQ])
{
    Real m[NQ];
    moments(K, f, m);
    const EqT<Real> q = equilibria(K, m[0], m[1], m[2], m[3]);
    const Real d5 = m[4] - q.e5, d6 = m[5] - q.e6, d7 = m[6] - q.e7, d8 = m[7] - q.e8;
    const Real d9 = m[8] - q.e9, d10 = m[9] - q.e10, d11 = m[10] - q.e11, d12 = m[11];
    const Real d13 = m[12] - q.e13, d14 = m[13] - q.e14, d15 = m[14], d16 = m[15];
    Real A[4], X[4], Y[4], Q[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        A[g] = fma_(K.c0[g][1], d12, K.c0[g][0] * d11);
        X[g] = fma_(K.cx[g][2], d15, fma_(K.cx[g][1], d9, K.cx[g][0] * d7));
        Y[g] = fma_(K.cy[g][2], d16, fma_(K.cy[g][1], d10, K.cy[g][0] * d8));
    }
    Q[0] = fma_(K.cqa[0][1], d13, K.cqa[0][0] * d5);
    Q[1] = fma_(K.cqa[1][1], d13, K.cqa[1][0] * d5);
    Q[2] = fma_(K.cqd[0][1], d14, K.cqd[0][0] * d6);
    Q[3] = fma_(K.cqd[1][1], d14, K.cqd[1][0] * d6);
    group_inv<true>(A[0], X[0], Y[0], Q[0], dC[0], dC[1], dC[2], dC[3]);
    group_inv<true>(A[1], X[1], Y[1], Q[1], dC[4], dC[5], dC[6], dC[7]);
    group_inv<false>(A[2], X[2], Y[2], Q[2], dC[8], dC[9], dC[10], dC[11]);
    group_inv<false>(A[3], X[3], Y[3], Q[3], dC[12], dC[13], dC[14], dC[15]);
}

// g^eq = M^-1 (f-hat^eq - f-hat_ref) from the conserved moments as
// deviations (dr = rho - rho0, j, de = e - e0): initial and boundary nodes.
template <class Real>
__device__ __forceinline__ void feq_of_moments(const ConstsT<Real> &K, Real dr, Real jx, Real jy,
                                               Real de, Real (&f)[NQ])
{
    const EqT<Real> q = equilibria(K, dr, jx, jy, de);
    const Real h0[4] = {dr, de, q.e11, Real(0.0)};
    const Real hx[4] = {jx, q.e7, q.e9, Real(0.0)};
    const Real hy[4] = {jy, q.e8, q.e10, Real(0.0)};
    Real A[4], X[4], Y[4], Q[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        A[g] = dot4(K.i0[g], h0);
        X[g] = dot4(K.ix[g], hx);
        Y[g] = dot4(K.iy[g], hy);
    }
    Q[0] = fma_(K.iqa[0][1], q.e13, K.iqa[0][0] * q.e5);
    Q[1] = fma_(K.iqa[1][1], q.e13, K.iqa[1][0] * q.e5);
    Q[2] = fma_(K.iqd[0][1], q.e14, K.iqd[0][0] * q.e6);
    Q[3] = fma_(K.iqd[1][1], q.e14, K.iqd[1][0] * q.e6);
    group_inv<true>(A[0], X[0], Y[0], Q[0], f[0], f[1], f[2], f[3]);
    group_inv<true>(A[1], X[1], Y[1], Q[1], f[4], f[5], f[6], f[7]);
    group_inv<false>(A[2], X[2], Y[2], Q[2], f[8], f[9], f[10], f[11]);
    group_inv<false>(A[3], X[3], Y[3], Q[3], f[12], f[13], f[14], f[15]);
}

// g^eq of a macroscopic state given as (rho - rho0, u1, u2, T - T0): initial
// and boundary nodes.  e - e0 = rho T - rho0 T0 + rho |u|^2 / 2 = rho0 (T - T0)
// + (rho - rho0) T + rho |u|^2 / 2.
template <class Real>
__device__ __forceinline__ void feq_velocity(const ConstsT<Real> &K, Real dr, Real ux, Real uy,
                                             Real dT, Real (&f)[NQ])
{
    const Real rho = K.rho0 + dr, T = K.T0 + dT;
    const Real jx = rho * ux, jy = rho * uy;
    const Real de = fma_(Real(0.5) * rho, fma_(ux, ux, uy * uy), fma_(dr, T, K.rho0 * dT));
    feq_of_moments(K, dr, jx, jy, de, f);
}

// (rho - rho0, u1, u2, T - T0) of one node's stored populations:
// T - T0 = (P - T0 rho) / rho = (de - T0 dr - |j|^2 / (2 rho)) / rho.
template <class Real>
__device__ __forceinline__ void macro_of(const ConstsT<Real> &K, const Real (&f)[NQ], Real (&q)[4])
{
    Real dr, jx, jy, de;
    conserved(K, f, dr, jx, jy, de);
    const Real r = Real(1.0) / (K.rho0 + dr);
    const Real ux = jx * r, uy = jy * r;
    const Real dP = fma_(-Real(0.5), jx * ux + jy * uy, fma_(-K.T0, dr, de));
    q[0] = dr;
    q[1] = ux;
    q[2] = uy;
    q[3] = dP * r;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x = hi + lo with both parts BF16 (|x - hi - lo| <= 2^-17 |x|).  The
// conversions round to nearest even (the packed hardware conversion of this
// target), as the host does for the constant operands.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef int i32x2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void split4(const float (&x)[4], bf16x4 &hi, bf16x4 &lo)
{
    i32x2v h, l;
#pragma unroll
    for (int p = 0; p < 2; ++p) {  // one packed conversion per pair
        const f32x2v v = {x[2 * p], x[2 * p + 1]};
        const bf16x2v hv = __builtin_convertvector(v, bf16x2v);
        const bf16x2v lv = __builtin_convertvector(v - __builtin_convertvector(hv, f32x2v), bf16x2v);
        h[p] = __builtin_bit_cast(int, hv);
        l[p] = __builtin_bit_cast(int, lv);
    }
    hi = __builtin_bit_cast(bf16x4, h);
    lo = __builtin_bit_cast(bf16x4, l);
}

// x = hi + mid + lo exactly, all three BF16: each remainder is exact in
// FP32 and the last one has at most 8 significant bits.
__device__ __forceinline__ void split4_exact(const float (&x)[4], bf16x4 &hi, bf16x4 &mid, bf16x4 &lo)
{
    i32x2v h, m, l;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const f32x2v v = {x[2 * p], x[2 * p + 1]};
        const bf16x2v hv = __builtin_convertvector(v, bf16x2v);
        const f32x2v r = v - __builtin_convertvector(hv, f32x2v);
        const bf16x2v mv = __builtin_convertvector(r, bf16x2v);
        const bf16x2v lv = __builtin_convertvector(r - __builtin_convertvector(mv, f32x2v), bf16x2v);
        h[p] = __builtin_bit_cast(int, hv);
        m[p] = __builtin_bit_cast(int, mv);
        l[p] = __builtin_bit_cast(int, lv);
    }
    hi = __builtin_bit_cast(bf16x4, h);
    mid = __builtin_bit_cast(bf16x4, m);
    lo = __builtin_bit_cast(bf16x4, l);
}

// The factored transform's 4x4 blocks on the matrix instruction
// v_mfma_f32_4x4x4_16b_bf16: lane l supplies row l % 4 of the block as A and
// its own node's 4 inputs as B, and receives the block's 4 outputs for its
// own node; FP32 accumulation.
//
// Forward blocks (exact BF16 weights, w.x and w.y = this lane's row packed):
// the inputs split exactly in three parts, smallest products first, so that
// the result is the FP32 dot product up to the accumulation's rounding.
__device__ __forceinline__ f32x4 block_fwd(uint4 w, const float (&x)[4])
{
    const bf16x4 wh = __builtin_bit_cast(bf16x4, make_uint2(w.x, w.y));
    bf16x4 xh, xm, xl;
    split4_exact(x, xh, xm, xl);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wh, xl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wh, xm, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wh, xh, c, 0, 0, 0);
    return c;
}

// Back-map blocks (weights dt s_k M^-1, not exact in BF16): w = (hi pair,
// hi pair, mid pair, mid pair) and w3 = (lo pair, lo pair, -, -) of this
// lane's row, hi + mid + lo = the FP32 weight exactly, so that the products
// carry no fixed bias of the relaxation rates; the inputs split in two.
// Four products, smallest first.  Left out: the weights' middle and low
// parts times the inputs' low parts (at most 2^-16 |w| |x|), and the inputs'
// own split remainder (at most 2^-17 |x|); both vary from node to node.
__device__ __forceinline__ f32x4 block_back(uint4 w, uint4 w3, const float (&x)[4])
{
    const bf16x4 wh = __builtin_bit_cast(bf16x4, make_uint2(w.x, w.y));
    const bf16x4 wm = __builtin_bit_cast(bf16x4, make_uint2(w.z, w.w));
    const bf16x4 wl = __builtin_bit_cast(bf16x4, make_uint2(w3.x, w3.y));
    bf16x4 xh, xl;
    split4(x, xh, xl);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wl, xh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wm, xh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wh, xl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(wh, xh, c, 0, 0, 0);
    return c;
}

// dC = dt * C of Eq. (3) with the moments and the back-map on the matrix
// cores (Bf3Ops: blocks 0-3 forward, 4-7 back, 8-11 the back blocks' third
// parts).  The forward blocks give all 16 moments, the conserved ones
// included, to FP32 accuracy; the back-map holds its weights exactly and
// splits its inputs, the nonequilibrium moments, into two BF16 parts (an
// error of at most 1.5 2^-16 of |dt s_k M^-1| times them).  The butterflies, the equilibria and the
// inverse butterfly stay FP32.  bt = the block table in LDS, row = lane % 4.
// Every lane of the wave must execute it.
__device__ __forceinline__ void collide_bf3(const Consts &K, const uint4 (*bt)[4], int row,
                                            const float (&f)[NQ], float (&dC)[NQ])
{
    // the table holds the diagonal groups' columns of fx and fy divided by
    // sqrt 2 (exact in BF16 then), so those inputs carry the factor
    constexpr float SQRT2 = 0x1.6a09e6p+0f;
    float A[4], X[4], Y[4], Q[4];
    butterflies(f, A, X, Y, Q);
    X[2] *= SQRT2;
    X[3] *= SQRT2;
    Y[2] *= SQRT2;
    Y[3] *= SQRT2;
    const f32x4 m0 = block_fwd(bt[0][row], A);  // rho - rho0, e - e0, m11, m12
    const f32x4 mx = block_fwd(bt[1][row], X);  // j_x, m7, m9, m15
    const f32x4 my = block_fwd(bt[2][row], Y);  // j_y, m8, m10, m16
    const f32x4 mq = block_fwd(bt[3][row], Q);  // m5, m13, m6, m14
    const EqT<float> q = equilibria(K, m0[0], mx[0], my[0], m0[1]);
    const float va[4] = {m0[2] - q.e11, m0[3], 0.f, 0.f};              // d11, d12
    const float vx[4] = {mx[1] - q.e7, mx[2] - q.e9, mx[3], 0.f};      // d7, d9, d15
    const float vy[4] = {my[1] - q.e8, my[2] - q.e10, my[3], 0.f};     // d8, d10, d16
    const float vq[4] = {mq[0] - q.e5, mq[1] - q.e13, mq[2] - q.e6, mq[3] - q.e14};  // d5, d13, d6, d14
    const f32x4 a = block_back(bt[4][row], bt[8][row], va);
    const f32x4 x = block_back(bt[5][row], bt[9][row], vx);
    const f32x4 y = block_back(bt[6][row], bt[10][row], vy);
    const f32x4 qq = block_back(bt[7][row], bt[11][row], vq);
    group_inv<true>(a[0], x[0], y[0], qq[0], dC[0], dC[1], dC[2], dC[3]);
    group_inv<true>(a[1], x[1], y[1], qq[1], dC[4], dC[5], dC[6], dC[7]);
    group_inv<false>(a[2], x[2], y[2], qq[2], dC[8], dC[9], dC[10], dC[11]);
    group_inv<false>(a[3], x[3], y[3], qq[3], dC[12], dC[13], dC[14], dC[15]);
}

// Which populations move along x / along y.
__host__ __device__ constexpr bool has_x(int q) { return q >= 8 || (q % 2) == 0; }
__host__ __device__ constexpr bool has_y(int q) { return q >= 8 || (q % 2) == 1; }

// Lax-Wendroff + Euler update of population q (same operation order in every
// kernel variant).  The step's increment (the four neighbour terms and the
// collision) is summed first and added to the node's value last, so that
// only that final addition rounds at the scale of the stored value; the
// others round at the scale of the increment.
template <int Q, class Real>
__device__ __forceinline__ Real lw_update(const ConstsT<Real> &K, Real fc, Real dC, Real fE, Real fW,
                                           Real fN, Real fS)
{
    Real r = -dC;
    if (has_x(Q)) {
        r = fma_(K.lw[Q][0], fE - fc, r);
        r = fma_(K.lw[Q][1], fW - fc, r);
    }
    if (has_y(Q)) {
        r = fma_(K.lw[Q][2], fN - fc, r);
        r = fma_(K.lw[Q][3], fS - fc, r);
    }
    return fc + r;
}

template <int Q>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F &&fn)
    {
        Unroll<Q - 1>::run(fn);
        fn(std::integral_constant<int, Q - 1>());
    }
};
template <>
struct Unroll<0> {
    template <class F>
    __device__ __forceinline__ static void run(F &&)
    {
    }
};

// ------------------------------------------------------------ boundary nodes

// Boundary nodes are never stored: a node next to a non-periodic side builds
// the value of its missing neighbour when it needs it ("virtual ghost"), and a
// periodic side is an index wrap.  The ghost node of side SD (0 west, 1 east,
// 2 south, 3 north) at along-side index a carries f^eq (stored as f^eq -
// f_ref) of a macroscopic state
// found by the side's rule (Sect. V) from n1, the boundary node itself, and n2,
// the next node inward, at time t.  The rule switches from kind_lo to kind_hi
// where the ghost's along-side coordinate passes split0 + split_rate t; that
// comparison is done in FP64.
template <int SD, class Real>
__device__ __forceinline__ void ghost_of(const ConstsT<Real> &K, const GhostsT<Real> &G, double t, int a,
                                         const Real (&n1)[NQ], const Real (&n2)[NQ],
                                         Real (&out)[NQ])
{
    const GhostSideT<Real> &S = G.side[SD];
    const double split = S.split0 + S.split_rate * t;
    const bool lo = ((double)a + 0.5) * S.h <= split;
    const int kind = lo ? S.kind_lo : S.kind_hi;
    if (kind == K_DIRICHLET) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] = lo ? S.feq_lo[q] : S.feq_hi[q];
        return;
    }
    Real q1[4], st[4];
    macro_of(K, n1, q1);
    if (kind == K_REFLECT) {
        st[0] = q1[0];
        st[1] = SD < 2 ? -q1[1] : q1[1];
        st[2] = SD < 2 ? q1[2] : -q1[2];
        st[3] = q1[3];
    } else if (kind == K_EXTRAPOLATE) {
        Real q2[4];
        macro_of(K, n2, q2);
#pragma unroll
        for (int c = 0; c < 4; ++c) st[c] = fma_(Real(2.0), q1[c], -q2[c]);
        if (!(K.rho0 + st[0] > Real(0.)) || !(K.T0 + st[3] > Real(0.))) {
#pragma unroll
            for (int c = 0; c < 4; ++c) st[c] = q1[c];
        }
    } else {  // wall: density of the fluid, speed and temperature of the wall (T - T0)
        st[0] = q1[0];
        st[1] = lo ? S.st_lo[1] : S.st_hi[1];
        st[2] = lo ? S.st_lo[2] : S.st_hi[2];
        st[3] = lo ? S.st_lo[3] : S.st_hi[3];
    }
    feq_velocity(K, st[0], st[1], st[2], st[3], out);
}

// ------------------------------------------------------------ step kernels

// Update of node (i, j) with its neighbours read from global memory, every
// boundary rule handled.  The Lax-Wendroff terms are added in the order east,
// west, north, south for every population, the order lw_update uses, so all
// kernel variants agree bit for bit.
template <class Real>
__device__ __forceinline__ void node_update(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                                            const Real *__restrict__ fin,
                                            Real *__restrict__ fout, int i, int j, double t)
{
    const int nx = F.nx, ny = F.ny;
    Real fc[NQ], out[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) fc[q] = fin[F.at(q, i, j)];
    {
        Real dC[NQ];
        collide(K, fc, dC);
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] = -dC[q];  // the increment, as in lw_update
    }
    if (i == nx - 1 && !G.per_x) {
        Real n2[NQ], g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) n2[q] = fin[F.at(q, i - 1, j)];
        ghost_of<1>(K, G, t, j, fc, n2, g);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_x(q)) out[q] = fma_(K.lw[q][0], g[q] - fc[q], out[q]);
    } else {
        const int ie = i == nx - 1 ? 0 : i + 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_x(q)) out[q] = fma_(K.lw[q][0], fin[F.at(q, ie, j)] - fc[q], out[q]);
    }
    if (i == 0 && !G.per_x) {
        Real n2[NQ], g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) n2[q] = fin[F.at(q, i + 1, j)];
        ghost_of<0>(K, G, t, j, fc, n2, g);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_x(q)) out[q] = fma_(K.lw[q][1], g[q] - fc[q], out[q]);
    } else {
        const int iw = i == 0 ? nx - 1 : i - 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_x(q)) out[q] = fma_(K.lw[q][1], fin[F.at(q, iw, j)] - fc[q], out[q]);
    }
    if (j == ny - 1 && !G.per_y) {
        Real n2[NQ], g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) n2[q] = fin[F.at(q, i, j - 1)];
        ghost_of<3>(K, G, t, i, fc, n2, g);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_y(q)) out[q] = fma_(K.lw[q][2], g[q] - fc[q], out[q]);
    } else {
        const int jn = j == ny - 1 ? 0 : j + 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_y(q)) out[q] = fma_(K.lw[q][2], fin[F.at(q, i, jn)] - fc[q], out[q]);
    }
    if (j == 0 && !G.per_y) {
        Real n2[NQ], g[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) n2[q] = fin[F.at(q, i, j + 1)];
        ghost_of<2>(K, G, t, i, fc, n2, g);
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_y(q)) out[q] = fma_(K.lw[q][3], g[q] - fc[q], out[q]);
    } else {
        const int js = j == 0 ? ny - 1 : j - 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_y(q)) out[q] = fma_(K.lw[q][3], fin[F.at(q, i, js)] - fc[q], out[q]);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) fout[F.at(q, i, j)] = fc[q] + out[q];
}

template <class Real>
__device__ __forceinline__ double step_time(const GhostsT<Real> &G, const long long *d_step, int k)
{
    return (double)(*d_step + k) * G.dt;
}

// One thread per node, 64x4 nodes per block; neighbours read straight from
// global memory (the caches absorb the re-reads).
template <class Real>
__global__ __launch_bounds__(256) void k_step_simple(Field F, ConstsT<Real> K, GhostsT<Real> G,
                                                     const Real *__restrict__ fin,
                                                     Real *__restrict__ fout,
                                                     const long long *__restrict__ d_step, int k)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= F.nx || j >= F.ny) return;
    node_update(F, K, G, fin, fout, i, j, step_time(G, d_step, k));
}

// Wavefront shifts across all 64 lanes (DPP wave_shr:1 / wave_shl:1, CDNA).
// shr1: lane l takes v from lane l-1, lane 0 keeps `edge`.
// shl1: lane l takes v from lane l+1, lane 63 keeps `edge`.
__device__ __forceinline__ float shr1(float v, float edge)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float shl1(float v, float edge)
{
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), 0x130, 0xF, 0xF, false));
}
// The same shifts of FP64 values: both 32-bit halves move by one lane.
__device__ __forceinline__ double shr1(double v, double edge)
{
    const int2 a = __builtin_bit_cast(int2, v), e = __builtin_bit_cast(int2, edge);
    const int2 r = make_int2(__builtin_amdgcn_update_dpp(e.x, a.x, 0x138, 0xF, 0xF, false),
                             __builtin_amdgcn_update_dpp(e.y, a.y, 0x138, 0xF, 0xF, false));
    return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double shl1(double v, double edge)
{
    const int2 a = __builtin_bit_cast(int2, v), e = __builtin_bit_cast(int2, edge);
    const int2 r = make_int2(__builtin_amdgcn_update_dpp(e.x, a.x, 0x130, 0xF, 0xF, false),
                             __builtin_amdgcn_update_dpp(e.y, a.y, 0x130, 0xF, 0xF, false));
    return __builtin_bit_cast(double, r);
}

// Buffer resource over one copy of f (raw buffer, byte offsets, 32-bit range
// checked by the hardware: out-of-range loads return 0, stores are dropped).
template <class Real>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const Real *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<Real *>(p), 0, (int)bytes, 0x00020000);
}
template <class Real = float>
__device__ __forceinline__ Real bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(Real) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    else
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, double v, unsigned voff, unsigned soff)
{
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0u, 0)) b64;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64, v), r, voff, soff, AUX);
}

// Row kernel.  Each wavefront updates R consecutive rows of 64 consecutive
// columns; the four waves of a block take vertically adjacent row groups of
// the same columns.  Rows y0-1 .. y0+R of the wave's columns are loaded once
// (the rows above and below only for populations moving in y), all loads
// issued before any arithmetic.  West/east neighbours come from the adjacent
// lanes by DPP; the two columns just outside the wave come from one extra
// load per population and row (lanes 0-31 read column x0-1, lanes 32-63
// column x0+64, so lane 0 and lane 63 hold what they need).  Addressing is by
// buffer instructions: one per-lane byte offset shared by all loads of a
// column, plus a wave-uniform offset for (plane, row).
//
// Waves at a side of the grid run the same steps in a branch of their own
// (rows_edge); what lies beyond the side is put into the registers that
// would hold the missing neighbours: on a
// periodic side the loads are redirected to the periodic image, otherwise
// the boundary ghost (ghost_of, the same function and inputs as node_update)
// replaces the south or north neighbour row, the west halo of lane 0, or the
// east neighbour of the last column (the halo of lane 63, or the values of
// the lane just past the last column, whose own result is not stored).  Only
// a wave whose last column is alone in it (nx = 1 mod 64), which has no
// second column for an east ghost, takes node_update.
//
// Real: the stored type, float or double (the FP64 mode: one row per wave,
// 64-bit buffer accesses and DPP shifts of both halves, two waves per SIMD
// with its 185 registers; held to three it spills and is slower).
// The row kernel's path for a wave at a side of the grid (see k_step_rows).
template <int R, int AUX, bool BF, class Real>
__device__ __forceinline__ void rows_edge(const Field &F, const ConstsT<Real> &K,
                                          const GhostsT<Real> &G, const Real *__restrict__ fin,
                                          Real *__restrict__ fout,
                                          unsigned bytes, int x0, int y0, int lane,
                                          const long long *__restrict__ d_step, int k,
                                          const uint4 (*bt)[4])
{
    const int nx = F.nx, ny = F.ny, x = x0 + lane;
    const bool west = x0 == 0, east = x0 + 64 >= nx;
    const bool south = y0 == 0, north = y0 + R >= ny;
    const int e = nx - 1 - x0;  // lane of the last column, when east
    // lanes past the last column read the periodic image on a periodic x side
    const int xl = (x >= nx && G.per_x) ? x - nx : x;
    int xh = lane < 32 ? x0 - 1 : x0 + 64;
    if (G.per_x && west && lane < 32) xh = nx - 1;
    if (G.per_x && east && e == 63 && lane >= 32) xh = 0;
    const unsigned vo = (unsigned)sizeof(Real) * (unsigned)F.col(xl);
    const unsigned vh = (unsigned)sizeof(Real) * (unsigned)F.col(xh);
    const unsigned es = (unsigned)sizeof(Real);
    const unsigned qB = es * (unsigned)F.qstride, jB = es * (unsigned)F.jstride;
    const auto rin = buffer_of(fin, bytes);
    const auto rout = buffer_of(fout, bytes);
    // byte offset of row j (j = -1 .. ny) of plane q
    auto row = [&](int q, int j) { return (unsigned)q * qB + (unsigned)(j + 1) * jB; };
    // rows -1 and ny of a periodic y side are the opposite edge rows
    auto jrow = [&](int j) { return !G.per_y ? j : j == -1 ? ny - 1 : j == ny ? 0 : j; };

    Real v[R + 2][NQ], h[R][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        v[0][q] = has_y(q) ? bload<Real>(rin, vo, row(q, jrow(y0 - 1))) : Real(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r + 1][q] = bload<Real>(rin, vo, row(q, jrow(y0 + r)));
            h[r][q] = has_x(q) ? bload<Real>(rin, vh, row(q, y0 + r)) : Real(0);
        }
        v[R + 1][q] = has_y(q) ? bload<Real>(rin, vo, row(q, jrow(y0 + R))) : Real(0);
    }
    const bool edge = (west && !G.per_x) || (east && !G.per_x) || (south && !G.per_y) ||
                      (north && !G.per_y);
    const double t = edge ? step_time(G, d_step, k) : 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = y0 + r;
        if (y >= ny) break;
        if (edge) {
            Real g[NQ], n2[NQ];
            if (y == 0 && !G.per_y) {  // south ghost replaces the row below
#pragma unroll
                for (int q = 0; q < NQ; ++q)  // row 1: a wave row when R > 1
                    n2[q] = (R > 1 || has_y(q)) ? v[r + 2][q] : bload<Real>(rin, vo, row(q, 1));
                ghost_of<2>(K, G, t, x, v[r + 1], n2, g);
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (has_y(q)) v[r][q] = g[q];
            }
            if (y == ny - 1 && !G.per_y) {  // north ghost replaces the row above
#pragma unroll
                for (int q = 0; q < NQ; ++q)  // row ny - 2: a wave row when r > 0
                    n2[q] = (r >= 1 || has_y(q)) ? v[r][q] : bload<Real>(rin, vo, row(q, ny - 2));
                ghost_of<3>(K, G, t, x, v[r + 1], n2, g);
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (has_y(q)) v[r + 2][q] = g[q];
            }
            if (west && !G.per_x) {  // west ghost: the halo of lane 0
#pragma unroll
                for (int q = 0; q < NQ; ++q) n2[q] = shl1(v[r + 1][q], Real(0));
                ghost_of<0>(K, G, t, y, v[r + 1], n2, g);
#pragma unroll
                for (int q = 0; q < NQ; ++q)
                    if (has_x(q) && lane == 0) h[r][q] = g[q];
            }
            if (east && !G.per_x) {
                if (e == 63) {  // east ghost: the halo of lane 63
#pragma unroll
                    for (int q = 0; q < NQ; ++q) n2[q] = shr1(v[r + 1][q], Real(0));
                    ghost_of<1>(K, G, t, y, v[r + 1], n2, g);
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (has_x(q) && lane == 63) h[r][q] = g[q];
                } else {  // east ghost: the values of the lane past the last column
                    Real n1[NQ];
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        n1[q] = shr1(v[r + 1][q], Real(0));
                        n2[q] = shr1(n1[q], Real(0));
                    }
                    ghost_of<1>(K, G, t, y, n1, n2, g);
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (x == nx) v[r + 1][q] = g[q];
                }
            }
        }
        Real dC[NQ];
        if constexpr (BF)
            collide_bf3(K, bt, lane & 3, v[r + 1], dC);
        else
            collide(K, v[r + 1], dC);
        Unroll<NQ>::run([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            Real fE = Real(0), fW = Real(0);
            if (has_x(q)) {
                fE = shl1(v[r + 1][q], h[r][q]);
                fW = shr1(v[r + 1][q], h[r][q]);
            }
            const Real o = lw_update<q>(K, v[r + 1][q], dC[q], fE, fW, v[r + 2][q], v[r][q]);
            if (x < nx) bstore<AUX>(rout, o, vo, row(q, y));
        });
    }
}

template <class Real>
__device__ __forceinline__ void face_flux_node(const Field &F, const ConstsT<Real> &K,
                                               const GhostsT<Real> &G, const FluxCoef &C,
                                               const Real *__restrict__ fin,
                                               double *__restrict__ slots,
                                               const long long *__restrict__ d_step, int k, int t);

// BUD: the first fblocks blocks (a multiple of 8, so that the XCD of every
// step block is unchanged) add the step's outflow budget from the input copy,
// one thread per side node, with the constants read from the device copies;
// dispatched first, they run beside the step blocks, which only write the
// other copy.
//
// BF: the collision's transforms in split-BF16 on the matrix cores
// (collide_bf3), its block table copied from bops into LDS first.
template <int R, int AUX, bool BUD, bool BF, class Real>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(Real) == 8 ? 2 : (R == 1 ? 5 : 3), 8)))
void k_step_rows(Field F, ConstsT<Real> K, GhostsT<Real> G, const Real *__restrict__ fin,
                 Real *__restrict__ fout, unsigned bytes, int ncol, int nrg, int nblocks,
                 const long long *__restrict__ d_step, int k, int order,
                 double *__restrict__ slots, int fblocks, const Bf3Ops *__restrict__ bops)
{
    int b = blockIdx.x;
    if (BUD) {
        if (b < fblocks) {
            face_flux_node(F, *G.kd, *G.gd, *G.fd, fin, slots, d_step, k,
                           b * 256 + (int)threadIdx.x);
            return;
        }
        b -= fblocks;
    }
    __shared__ uint4 bt[BF ? 12 : 1][4];
    if (BF) {  // every thread of the block reaches this barrier
        if (threadIdx.x < 48) bt[threadIdx.x >> 2][threadIdx.x & 3] = bops->w[threadIdx.x >> 2][threadIdx.x & 3];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Consecutive blocks land on different XCDs (round robin over 8); give
    // each XCD a contiguous range of tiles so that neighbouring tiles, which
    // share halo rows and columns, share an L2: a band of whole tile rows
    // (order 0), or of ncol/8 tile columns (order 1, taken when the tile
    // columns and blocks divide by 8).
    if ((nblocks & 7) == 0) b = (b & 7) * (nblocks >> 3) + (b >> 3);
    int col, rb;
    if (order == 1) {
        const int cw = ncol >> 3, nrb = nblocks / ncol;
        col = (b / (nrb * cw)) * cw + b % cw;
        rb = (b / cw) % nrb;
    } else {
        col = b % ncol;
        rb = b / ncol;
    }
    const int rg = rb * 4 + wv;
    if (rg >= nrg) return;
    const int x0 = col * 64, y0 = rg * R, x = x0 + lane;
    if (col == 0 || x0 + 64 >= F.nx || y0 == 0 || y0 + R >= F.ny) {
        // constants from the device copies (see Ghosts::kd)
        const ConstsT<Real> &Kd = *G.kd;
        const GhostsT<Real> &Gd = *G.gd;
        if (x0 + 1 == F.nx) {  // a last column alone in its wave
            const double t = step_time(Gd, d_step, k);
            if (x < F.nx) {
#pragma unroll 1
                for (int r = 0; r < R; ++r)
                    if (y0 + r < F.ny) node_update(F, Kd, Gd, fin, fout, x, y0 + r, t);
            }
        } else {
            rows_edge<R, AUX, BF, Real>(F, Kd, Gd, fin, fout, bytes, x0, y0, lane, d_step, k, bt);
        }
        return;
    }
    const unsigned vo = (unsigned)sizeof(Real) * (unsigned)F.col(x);
    const unsigned vh = (unsigned)sizeof(Real) * (unsigned)F.col(lane < 32 ? x0 - 1 : x0 + 64);
    const unsigned es = (unsigned)sizeof(Real);
    const unsigned qB = es * (unsigned)F.qstride, jB = es * (unsigned)F.jstride;
    const auto rin = buffer_of(fin, bytes);
    const auto rout = buffer_of(fout, bytes);
    // byte offset of row j (j = -1 .. ny) of plane q
    auto row = [&](int q, int j) { return (unsigned)q * qB + (unsigned)(j + 1) * jB; };

    Real v[R + 2][NQ], h[R][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        v[0][q] = has_y(q) ? bload<Real>(rin, vo, row(q, y0 - 1)) : Real(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r + 1][q] = bload<Real>(rin, vo, row(q, y0 + r));
            h[r][q] = has_x(q) ? bload<Real>(rin, vh, row(q, y0 + r)) : Real(0);
        }
        v[R + 1][q] = has_y(q) ? bload<Real>(rin, vo, row(q, y0 + R)) : Real(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        Real dC[NQ];
        if constexpr (BF)
            collide_bf3(K, bt, lane & 3, v[r + 1], dC);
        else
            collide(K, v[r + 1], dC);
        Unroll<NQ>::run([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            Real fE = Real(0), fW = Real(0);
            if (has_x(q)) {
                fE = shl1(v[r + 1][q], h[r][q]);
                fW = shr1(v[r + 1][q], h[r][q]);
            }
            const Real o = lw_update<q>(K, v[r + 1][q], dC[q], fE, fW, v[r + 2][q], v[r][q]);
            bstore<AUX>(rout, o, vo, row(q, y0 + r));
        });
    }
}

// ------------------------------------------------------------- tube batches

// Temporal blocking of one work item (columns [x0, x0 + S) of a tube) over KS
// steps.  The block covers the 4 rows of columns x0 - KS .. x0 + S + KS - 1
// (64 columns: one wave per row, one lane per column) and keeps each node's
// 16 populations in registers for the whole round: west/east neighbours come
// from the adjacent lanes by DPP, north/south neighbours (the rows are
// periodic) from the other waves through LDS, where each step publishes the
// populations that move in y.  After each step the outermost valid column on
// each side goes stale (a trapezoid), except at the ends of the tube, where
// the column beyond the end holds the constant boundary equilibrium for every
// step.  After the last step the S owned columns are written back.  Each
// node's update is the same arithmetic as the single-grid kernels (collide,
// then the east/west/north/south terms in that order), so a tube run here
// equals the same tube run as a grid, bit for bit.
__host__ __device__ constexpr int yslot(int q) { return q < 8 ? q >> 1 : q - 4; }  // has_y(q)

template <int S, int KS>
__global__ __launch_bounds__(256) void k_tubes(TubeGrid TG, const Consts *__restrict__ Kd,
                                               const TubeInfo *__restrict__ tubes,
                                               const TubeItem *__restrict__ items, int round,
                                               const float *__restrict__ fin,
                                               float *__restrict__ fout)
{
    constexpr int TW = S + 2 * KS;
    constexpr int WY = TUBE_ROWS;
    static_assert(TW == 64 && WY * 64 == 256, "one wave per row, one lane per column");
    __shared__ float ybuf[2][12][WY][TW];  // y-moving populations, by step parity
    const TubeItem it = items[blockIdx.x];
    const int n = tubes[it.tube].n;
    const int start = tubes[it.tube].start;
    const int nsteps = min(KS, tubes[it.tube].steps - round * KS);
    const int xbase = it.x0 - KS;  // tube column of tile column 0
    const int cL = -1 - xbase;     // tile column of the west boundary node (x = -1)
    const int cR = n - xbase;      // tile column of the east boundary node (x = n)
    const int y = threadIdx.x >> 6, c = threadIdx.x & 63;
    const int yn = y == WY - 1 ? 0 : y + 1, ys = y == 0 ? WY - 1 : y - 1;
    const int x = xbase + c;
    const long long base = (long long)y * TG.ncols + start + x;
    float f[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        float v = 0.f;
        if (x >= 0 && x < n)
            v = fin[(long long)q * TG.plane + base];
        else if (x == -1)
            v = tubes[it.tube].feq_left[q];
        else if (x == n)
            v = tubes[it.tube].feq_right[q];
        f[q] = v;
    }
    for (int st = 0; st < nsteps; ++st) {
        // valid input columns [a, b); update a+1 .. b-2 (interior nodes only)
        const int a = cL >= 0 ? cL : st;
        const int b = cR < TW ? cR + 1 : TW - st;
        const bool upd = c > a && c < b - 1;
        float(*yb)[WY][TW] = ybuf[st & 1];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (has_y(q)) yb[yslot(q)][y][c] = f[q];
        __syncthreads();
        // The constants are read from memory in every step: held across the
        // loop they exceed the scalar registers and spill to vector lanes.
        unsigned long long ka = reinterpret_cast<unsigned long long>(Kd);
        asm volatile("" : "+s"(ka));
        typedef const __attribute__((address_space(4))) Consts ConstConsts;
        const Consts &K = *(const Consts *)(ConstConsts *)ka;
        float dC[NQ], g[NQ];
        collide(K, f, dC);
        Unroll<NQ>::run([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            float fE = 0.f, fW = 0.f, fN = 0.f, fS = 0.f;
            if (has_x(q)) {  // lanes 0 and 63 are never updated
                fE = shl1(f[q], 0.f);
                fW = shr1(f[q], 0.f);
            }
            if (has_y(q)) {
                fN = yb[yslot(q)][yn][c];
                fS = yb[yslot(q)][ys][c];
            }
            g[q] = lw_update<q>(K, f[q], dC[q], fE, fW, fN, fS);
        });
#pragma unroll
        for (int q = 0; q < NQ; ++q) f[q] = upd ? g[q] : f[q];
    }
    if (c >= KS && c < KS + S && x >= 0 && x < n) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) fout[(long long)q * TG.plane + base] = f[q];
    }
}

__global__ __launch_bounds__(256) void k_tubes_init(TubeGrid TG, Consts K,
                                                    const TubeInfo *__restrict__ tubes,
                                                    const float *__restrict__ states,
                                                    float *__restrict__ f)
{
    const int k = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int n = tubes[k].n;
    if (x >= n) return;
    const float *st = states + (long long)k * 8 + (x < n / 2 ? 0 : 4);
    float fe[NQ];
    feq_velocity(K, st[0] - K.rho0, st[1], st[2], st[3] - K.T0, fe);
    const int start = tubes[k].start;
    for (int y = 0; y < TUBE_ROWS; ++y)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            f[(long long)q * TG.plane + (long long)y * TG.ncols + start + x] = fe[q];
}

__global__ __launch_bounds__(256) void k_tube_macro(TubeGrid TG, Consts K,
                                                    const TubeInfo *__restrict__ tubes, int k,
                                                    const float *__restrict__ f, float *rho,
                                                    float *ux, float *uy, float *Tt, float *p)
{
    const int n = tubes[k].n, start = tubes[k].start;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n * TUBE_ROWS) return;
    const int y = idx / n, x = idx % n;
    float fc[NQ], q[4];
#pragma unroll
    for (int c = 0; c < NQ; ++c) fc[c] = f[(long long)c * TG.plane + (long long)y * TG.ncols + start + x];
    macro_of(K, fc, q);
    const float rh = K.rho0 + q[0], tt = K.T0 + q[3];
    if (rho) rho[idx] = rh;
    if (ux) ux[idx] = q[1];
    if (uy) uy[idx] = q[2];
    if (Tt) Tt[idx] = tt;
    if (p) p[idx] = rh * tt;
}

__global__ __launch_bounds__(256) void k_tube_pack(TubeGrid TG, const TubeInfo *__restrict__ tubes,
                                                   int k, const float *__restrict__ f,
                                                   float *__restrict__ dst)
{
    const int n = tubes[k].n, start = tubes[k].start;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (idx >= n * TUBE_ROWS) return;
    const int y = idx / n, x = idx % n;
    dst[(long long)q * n * TUBE_ROWS + idx] = f[(long long)q * TG.plane + (long long)y * TG.ncols + start + x];
}

// ------------------------------------------------------------ other kernels

template <class Real>
__global__ __launch_bounds__(256) void k_init(Field F, ConstsT<Real> K, Real *__restrict__ f,
                                              const float *__restrict__ rho,
                                              const float *__restrict__ ux,
                                              const float *__restrict__ uy,
                                              const float *__restrict__ T, int *flag)
{
    const long long n = (long long)F.nx * F.ny;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % F.nx), j = (int)(c / F.nx);
    const float r = rho[c], t = T[c];
    if (!(r > 0.f) || !(t > 0.f) || !isfinite(ux[c]) || !isfinite(uy[c]) || !isfinite(r) ||
        !isfinite(t))
        atomicOr(flag, 1);
    Real fe[NQ];
    feq_velocity(K, Real(r) - K.rho0, Real(ux[c]), Real(uy[c]), Real(t) - K.T0, fe);
#pragma unroll
    for (int q = 0; q < NQ; ++q) f[F.at(q, i, j)] = fe[q];
}

// Fill n 16-byte words, then `tail` 4-byte words after them, with the 32-bit
// pattern v (grid-stride).  Used instead of memset nodes, so that a caller may
// capture the calls that clear memory into a graph.
__global__ __launch_bounds__(256) void k_fill(uint4 *p, size_t n, unsigned *tail, int ntail,
                                              unsigned v)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        p[i] = make_uint4(v, v, v, v);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = v;
}

__global__ void k_counter(long long *d_step, long long n, int set)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (set)
            d_step[0] = n;
        else
            d_step[0] += n;
    }
}

// Readout in the stored precision, written as FP32 fields.
template <class Real>
__global__ __launch_bounds__(256) void k_read_macro(Field F, ConstsT<Real> K,
                                                    const Real *__restrict__ f, float *rho,
                                                    float *ux, float *uy, float *T, float *p)
{
    const long long n = (long long)F.nx * F.ny;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int i = (int)(c % F.nx), j = (int)(c / F.nx);
    Real fc[NQ], q[4];
#pragma unroll
    for (int k = 0; k < NQ; ++k) fc[k] = f[F.at(k, i, j)];
    macro_of(K, fc, q);
    const Real rh = K.rho0 + q[0], tt = K.T0 + q[3];
    if (rho) rho[c] = (float)rh;
    if (ux) ux[c] = (float)q[1];
    if (uy) uy[c] = (float)q[2];
    if (T) T[c] = (float)tt;
    if (p) p[c] = (float)(rh * tt);
}


// FP64 sums of rho, j_x, j_y, e.  Each thread walks a fixed set of nodes,
// then a fixed-order tree reduction per block; a second kernel adds the block
// partials in order.  The result is independent of timing.
template <class Real>
__global__ __launch_bounds__(256) void k_sums_partial(Field F, SumW W, const Real *__restrict__ f,
                                                      double *partials)
{
    __shared__ double sh[4][256];
    const long long n = (long long)F.nx * F.ny;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n;
         c += (long long)gridDim.x * 256) {
        const int i = (int)(c % F.nx), j = (int)(c / F.nx);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double v = (double)f[F.at(q, i, j)];
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += W.w[k][q] * v;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_sums_final(const double *__restrict__ partials, int nblk,
                                                    SumW W, double *out)
{
    __shared__ double sh[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += partials[b * 4 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[threadIdx.x] = sh[threadIdx.x][0] + W.add[threadIdx.x];
}

// Outflow budget.  One thread per node next to a side (west rows, east
// rows, south columns, north columns).  The node beyond the side is the
// boundary ghost (same rule and clock as the step) or, on a periodic side,
// the periodic image; the face value of the Lax-Wendroff difference between
// the two nodes, weighted by the conserved moments, is taken in FP64 from
// the FP32 populations and added to the thread's own slot, so the totals do
// not depend on scheduling.  Periodic faces are counted on both sides with
// equal and opposite values.
template <class Real>
__device__ __forceinline__ void face_flux_node(const Field &F, const ConstsT<Real> &K,
                                               const GhostsT<Real> &G, const FluxCoef &C,
                                               const Real *__restrict__ fin,
                                               double *__restrict__ slots,
                                               const long long *__restrict__ d_step, int k, int t)
{
    const int nx = F.nx, ny = F.ny;
    if (t >= 2 * (nx + ny)) return;
    int sd, a;
    if (t < ny) {
        sd = 0, a = t;
    } else if (t < 2 * ny) {
        sd = 1, a = t - ny;
    } else if (t < 2 * ny + nx) {
        sd = 2, a = t - 2 * ny;
    } else {
        sd = 3, a = t - 2 * ny - nx;
    }
    // first and second interior node along the inward normal
    int i1, j1, i2, j2;
    if (sd == 0) i1 = 0, i2 = 1, j1 = j2 = a;
    else if (sd == 1) i1 = nx - 1, i2 = nx - 2, j1 = j2 = a;
    else if (sd == 2) j1 = 0, j2 = 1, i1 = i2 = a;
    else j1 = ny - 1, j2 = ny - 2, i1 = i2 = a;
    Real n1[NQ], n2[NQ], g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) n1[q] = fin[F.at(q, i1, j1)];
    const bool per = sd < 2 ? G.per_x : G.per_y;
    if (per) {
        const int io = sd == 0 ? nx - 1 : sd == 1 ? 0 : a;
        const int jo = sd == 2 ? ny - 1 : sd == 3 ? 0 : a;
#pragma unroll
        for (int q = 0; q < NQ; ++q) g[q] = fin[F.at(q, io, jo)];
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) n2[q] = fin[F.at(q, i2, j2)];
        const double tm = step_time(G, d_step, k);
        if (sd == 0) ghost_of<0>(K, G, tm, a, n1, n2, g);
        else if (sd == 1) ghost_of<1>(K, G, tm, a, n1, n2, g);
        else if (sd == 2) ghost_of<2>(K, G, tm, a, n1, n2, g);
        else ghost_of<3>(K, G, tm, a, n1, n2, g);
    }
    // west/south: the ghost is at the lower coordinate and outflow is -phi
    const bool low_side = sd == 0 || sd == 2;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (!(sd < 2 ? has_x(q) : has_y(q))) continue;
        const double c0 = sd < 2 ? C.cx[q][0] : C.cy[q][0];
        const double c1 = sd < 2 ? C.cx[q][1] : C.cy[q][1];
        const double lo = low_side ? (double)g[q] : (double)n1[q];
        const double hi = low_side ? (double)n1[q] : (double)g[q];
        const double phi = c0 * (lo + hi) - c1 * (hi - lo);
        const double o = low_side ? -phi : phi;
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] += C.w[m][q] * o;
    }
    double *sl = slots + 4 * (long long)t;
#pragma unroll
    for (int m = 0; m < 4; ++m) sl[m] += acc[m];
}

template <class Real>
__global__ __launch_bounds__(256) void k_face_flux(Field F, ConstsT<Real> K, GhostsT<Real> G,
                                                   FluxCoef C, const Real *__restrict__ fin,
                                                   double *__restrict__ slots,
                                                   const long long *__restrict__ d_step, int k)
{
    face_flux_node(F, K, G, C, fin, slots, d_step, k, blockIdx.x * 256 + threadIdx.x);
}

// Per-side totals of the slots, one block per side, fixed summation order.
__global__ __launch_bounds__(256) void k_flux_totals(int nx, int ny,
                                                     const double *__restrict__ slots,
                                                     double *__restrict__ out)
{
    __shared__ double sh[4][256];
    const int sd = blockIdx.x;
    const int n = sd < 2 ? ny : nx;
    const int off = sd == 0 ? 0 : sd == 1 ? ny : sd == 2 ? 2 * ny : 2 * ny + nx;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < n; i += 256) {
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] += slots[4 * (long long)(off + i) + m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] = acc[m];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) out[4 * sd + threadIdx.x] = sh[threadIdx.x][0];
}

template <class Src, class Dst>
__global__ __launch_bounds__(256) void k_pack(Field F, const Src *__restrict__ f,
                                              Dst *__restrict__ dst)
{
    const long long n = (long long)F.nx * F.ny;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (c >= n) return;
    const int i = (int)(c % F.nx), j = (int)(c / F.nx);
    dst[(long long)q * n + c] = (Dst)f[F.at(q, i, j)];
}

template <class Src, class Dst>
__global__ __launch_bounds__(256) void k_unpack(Field F, const Src *__restrict__ src,
                                                Dst *__restrict__ f)
{
    const long long n = (long long)F.nx * F.ny;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    const int q = blockIdx.y;
    if (c >= n) return;
    const int i = (int)(c % F.nx), j = (int)(c / F.nx);
    f[F.at(q, i, j)] = (Dst)src[(long long)q * n + c];
}

// Von Neumann screen: all 16 eigenvalues of the amplification matrix G of
// Sect. IV for one phase pair per group of 16 lanes (four per wave), FP64
// complex (double2 = re, im) in LDS.  G is first balanced (Parlett and
// Reinsch 1969: row and column i scaled by powers of 2, which is exact,
// until their 1-norms are within a factor 2), then brought to upper
// Hessenberg form by Householder reflections, then reduced by the shifted
// QR algorithm (Francis 1961; Golub and Van Loan, Matrix Computations,
// Sect. 7.5) on the active window only, since only the eigenvalues are
// wanted: each step takes the Wilkinson shift of the trailing 2 x 2 block
// (an ad hoc shift every 10th step without deflation), factors H - mu I by
// Givens rotations, forms R Q + mu I, and deflates a subdiagonal entry once
// it is below the unit roundoff times its two diagonal neighbours.  The 16
// lanes of a group compute the same control flow and rotation scalars from
// the same LDS values, so branches are uniform within a group; groups share
// nothing, and a group's lanes order their LDS accesses by wave-scope
// fences (one wave executes its LDS instructions in order).
constexpr int SCREEN_GROUP = 16;                     // lanes per matrix
constexpr int SCREEN_PER_BLOCK = 64 / SCREEN_GROUP;  // matrices per wave (one wave per block)
constexpr int SCREEN_MAX_STEPS = 30 * NQ;

__device__ inline double2 c_mul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ inline double2 c_conj_mul(double2 a, double2 b)  // conj(a) * b
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.x, b.y, -a.y * b.x));
}
__device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 c_scale(double2 a, double r) { return make_double2(a.x * r, a.y * r); }
__device__ inline double c_abs1(double2 a) { return fabs(a.x) + fabs(a.y); }
__device__ inline double c_abs(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 c_div(double2 a, double2 b)  // Smith's algorithm
{
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, d = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    }
    const double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ inline double2 c_sqrt(double2 z)  // principal root, no cancellation
{
    const double r = c_abs(z);
    if (r == 0.0) return make_double2(0.0, 0.0);
    if (z.x >= 0.0) {
        const double t = sqrt(0.5 * (r + z.x));
        return make_double2(t, z.y / (2.0 * t));
    }
    const double t = sqrt(0.5 * (r - z.x));
    return make_double2(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 16 lanes of a group by a fixed butterfly: every lane gets the
// same bits (each addition pairs the same two values, and + commutes).
__device__ inline double group_sum(double x)
{
    x += __shfl_xor(x, 8, SCREEN_GROUP);
    x += __shfl_xor(x, 4, SCREEN_GROUP);
    x += __shfl_xor(x, 2, SCREEN_GROUP);
    x += __shfl_xor(x, 1, SCREEN_GROUP);
    return x;
}

// Givens rotation [[c, s], [-conj(s), c]] (c real) that zeroes b against a:
// c = |a| / r, s = conj(b) a / (|a| r), r = sqrt(|a|^2 + |b|^2), with a and b
// first scaled exactly by the power of 2 that brings max(|a|_1, |b|_1) into
// [1/2, 1), so that no square under- or overflows; a = 0 gives the swap (0,
// 1), a = b = 0 the identity.
__device__ inline void givens(double2 a, double2 b, double &c, double2 &s)
{
    const double m = fmax(c_abs1(a), c_abs1(b));
    if (m == 0.0) {
        c = 1.0;
        s = make_double2(0.0, 0.0);
        return;
    }
    int e;
    frexp(m, &e);
    a = make_double2(ldexp(a.x, -e), ldexp(a.y, -e));
    b = make_double2(ldexp(b.x, -e), ldexp(b.y, -e));
    const double na2 = a.x * a.x + a.y * a.y, r2 = na2 + b.x * b.x + b.y * b.y;
    if (na2 < 0x1p-1000) {  // |a| below 2^-500 |b|: a rotation by pi / 2 leaves at most |a| behind
        c = 0.0;
        s = make_double2(1.0, 0.0);
        return;
    }
    const double rinv = rsqrt(na2 * r2);  // 1 / (|a| r)
    c = na2 * rinv;
    s = c_scale(c_conj_mul(b, a), rinv);
}

// LDS of one wave's four matrices.
struct ScreenLds {
    double2 A[SCREEN_PER_BLOCK][NQ][NQ];
    double2 v[SCREEN_PER_BLOCK][NQ], w[SCREEN_PER_BLOCK][NQ];
    double rc[SCREEN_PER_BLOCK][NQ], mod[SCREEN_PER_BLOCK][NQ];
    double2 rs[SCREEN_PER_BLOCK][NQ], ev[SCREEN_PER_BLOCK][NQ];
};

// Lax-Wendroff factor of velocity i at the phases (tx, ty), Eq. (A.1b):
// 1 - i a sin(tx) + a^2 (cos(tx) - 1) - i b sin(ty) + b^2 (cos(ty) - 1).
__device__ inline double2 lw_factor(double a, double b, double tx, double ty)
{
    return make_double2(1.0 + a * a * (cos(tx) - 1.0) + b * b * (cos(ty) - 1.0), -(a * sin(tx) + b * sin(ty)));
}

// The eigenvalues of group g's matrix in L.A[g] (its lane t calling):
// balancing, Householder reduction, shifted QR, then the ranking by modulus.
// Lane t returns the eigenvalue e of rank `rank` (largest modulus first, ties
// by index) and its modulus m; all NaN, ranked by lane, when the iteration
// does not converge or any eigenvalue is NaN.
__device__ void screen_eig(ScreenLds &L, int g, int t, double2 &e_out, double &m_out, int &rank_out)
{
    auto &A = L.A[g];
    double2 *v = L.v[g], *w = L.w[g], *rs = L.rs[g], *ev = L.ev[g];
    double *rc = L.rc[g], *mod = L.mod[g];

    // balancing
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool changed = false;
        for (int i = 0; i < NQ; ++i) {
            double c = group_sum(t != i ? c_abs1(A[t][i]) : 0.0);
            const double r = group_sum(t != i ? c_abs1(A[i][t]) : 0.0);
            if (!(c > 0.0 && r > 0.0 && isfinite(c + r))) continue;
            const double s0 = c + r;
            double f = 1.0;
            for (int k = 0; k < 1000 && c < 0.5 * r; ++k) {
                f *= 2.0;
                c *= 4.0;
            }
            for (int k = 0; k < 1000 && c >= 2.0 * r; ++k) {
                f *= 0.5;
                c *= 0.25;
            }
            if ((c + r) / f < 0.95 * s0) {  // c is now c f^2: new column + row norm < 0.95 old
                changed = true;
                wave_sync();
                if (t != i) {
                    A[i][t] = c_scale(A[i][t], 1.0 / f);
                    A[t][i] = c_scale(A[t][i], f);
                }
                wave_sync();
            }
        }
        if (!changed) break;
    }

    // Householder reduction to upper Hessenberg form
    for (int k = 0; k + 2 < NQ; ++k) {
        const double2 xt = A[t][k];
        const double tail = group_sum(t >= k + 2 ? xt.x * xt.x + xt.y * xt.y : 0.0);
        if (tail == 0.0) continue;
        const double2 x0 = A[k + 1][k];
        const double a0 = c_abs(x0);
        const double xn = sqrt(tail + a0 * a0);
        const double2 ph = a0 > 0.0 ? c_scale(x0, 1.0 / a0) : make_double2(1.0, 0.0);
        const double2 alpha = c_scale(ph, -xn);           // v = x - alpha e_1: no cancellation in v_0
        const double tau = 1.0 / (xn * (xn + a0));        // 2 / (v^H v)
        if (t > k) v[t] = t == k + 1 ? c_scale(ph, a0 + xn) : xt;
        wave_sync();
        if (t > k) {  // w_t = v^H A(:, t) over rows k + 1 ..
            double2 acc = make_double2(0.0, 0.0);
            for (int i = k + 1; i < NQ; ++i) acc = c_add(acc, c_conj_mul(v[i], A[i][t]));
            w[t] = acc;
        }
        wave_sync();
        if (t == k)
            for (int r = k + 1; r < NQ; ++r) A[r][k] = r == k + 1 ? alpha : make_double2(0.0, 0.0);
        else if (t > k)
            for (int r = k + 1; r < NQ; ++r) A[r][t] = c_sub(A[r][t], c_scale(c_mul(v[r], w[t]), tau));
        wave_sync();
        {  // z_t = A(t, :) v over columns k + 1 ..
            double2 acc = make_double2(0.0, 0.0);
            for (int j = k + 1; j < NQ; ++j) acc = c_add(acc, c_mul(A[t][j], v[j]));
            wave_sync();
            w[t] = acc;
        }
        wave_sync();
        if (t > k) {
            const double2 vc = make_double2(v[t].x, -v[t].y);
            for (int r = 0; r < NQ; ++r) A[r][t] = c_sub(A[r][t], c_scale(c_mul(w[r], vc), tau));
        }
        wave_sync();
    }

    // shifted QR on the active window [l, hi]
    const double ulp = 0x1p-52;
    int hi = NQ - 1, since = 0, steps = 0;
    bool failed = false;
    while (hi >= 0) {
        bool small = false;
        if (t >= 1 && t <= hi) {
            const double sub = c_abs1(A[t][t - 1]);
            small = sub <= ulp * (c_abs1(A[t - 1][t - 1]) + c_abs1(A[t][t])) || sub < 0x1p-1000;
        }
        const unsigned mask = (unsigned)(__ballot(small) >> (SCREEN_GROUP * g)) & 0xffffu;
        const int l = mask ? 31 - __clz(mask) : 0;  // the last negligible subdiagonal entry at or above hi
        if (l == hi) {
            if (t == 0) ev[hi] = A[hi][hi];
            --hi;
            since = 0;
            continue;
        }
        if (steps == SCREEN_MAX_STEPS) {
            failed = true;
            break;
        }
        ++steps;
        ++since;
        double2 mu;
        if (since % 10 == 0) {
            mu = A[hi][hi];
            mu.x += 0.75 * c_abs1(A[hi][hi - 1]);
        } else {
            const double2 a = A[hi - 1][hi - 1], b = A[hi - 1][hi], c = A[hi][hi - 1], d = A[hi][hi];
            const double2 h = c_scale(c_sub(a, d), 0.5), bc = c_mul(b, c);
            const double2 root = c_sqrt(c_add(c_mul(h, h), bc));
            const double2 d1 = c_add(h, root), d2 = c_sub(h, root);
            const double2 den = c_abs1(d1) >= c_abs1(d2) ? d1 : d2;
            mu = c_abs1(den) > 0.0 ? c_sub(d, c_div(bc, den)) : d;
        }
        wave_sync();
        if (t >= l && t <= hi) A[t][t] = c_sub(A[t][t], mu);
        wave_sync();
        for (int k = l; k < hi; ++k) {  // H - mu I = Q R, rotation k zeroes (k + 1, k)
            double cr;
            double2 sr;
            givens(A[k][k], A[k + 1][k], cr, sr);
            wave_sync();
            if (t == 0) {
                rc[k] = cr;
                rs[k] = sr;
            }
            if (t >= k && t <= hi) {
                const double2 x = A[k][t], y = A[k + 1][t];
                A[k][t] = c_add(c_scale(x, cr), c_mul(sr, y));
                A[k + 1][t] = c_sub(c_scale(y, cr), c_conj_mul(sr, x));
            }
            wave_sync();
        }
        for (int k = l; k < hi; ++k) {  // R Q: columns k, k + 1 times the rotation's adjoint
            const double cr = rc[k];
            const double2 sr = rs[k];
            if (t >= l && t <= min(k + 1, hi)) {
                const double2 x = A[t][k], y = A[t][k + 1];
                A[t][k] = c_add(c_scale(x, cr), c_mul(y, make_double2(sr.x, -sr.y)));
                A[t][k + 1] = c_sub(c_scale(y, cr), c_mul(x, sr));
            }
            wave_sync();
        }
        if (t >= l && t <= hi) A[t][t] = c_add(A[t][t], mu);
        wave_sync();
    }
    wave_sync();
    // largest modulus first: lane t places its eigenvalue at its rank (ties by index)
    double2 e = failed ? make_double2(NAN, NAN) : ev[t];
    double m = failed ? NAN : c_abs(e);
    if ((__ballot(isnan(m)) >> (SCREEN_GROUP * g)) & 0xffffu) {  // NaN anywhere: all NaN, in lane order
        e = make_double2(NAN, NAN);
        m = NAN;
    }
    mod[t] = m;
    wave_sync();
    int rank = 0;
    for (int j = 0; j < NQ; ++j) {
        const double mj = mod[j];
        rank += (mj > m || (mj == m && j < t)) ? 1 : 0;
    }
    if (isnan(m)) rank = t;
    e_out = e;
    m_out = m;
    rank_out = rank;
}

__global__ __launch_bounds__(64) void k_screen(ScreenCoef S, const double *__restrict__ theta, int n,
                                               double *__restrict__ eig, double *__restrict__ rho)
{
    __shared__ ScreenLds L;
    const int g = threadIdx.x / SCREEN_GROUP, t = threadIdx.x % SCREEN_GROUP;
    const int p = blockIdx.x * SCREEN_PER_BLOCK + g;
    if (p >= n) return;  // the whole group
    const double tx = theta[2 * p], ty = theta[2 * p + 1];
    for (int r = 0; r < NQ; ++r) {  // lane t builds column t
        double2 e = make_double2(-S.C[r][t], 0.0);
        if (r == t) e = c_add(e, lw_factor(S.a[r], S.b[r], tx, ty));
        L.A[g][r][t] = e;
    }
    wave_sync();
    double2 e;
    double m;
    int rank;
    screen_eig(L, g, t, e, m, rank);
    if (eig) {
        eig[(long long)p * 2 * NQ + 2 * rank] = e.x;
        eig[(long long)p * 2 * NQ + 2 * rank + 1] = e.y;
    }
    if (rho && rank == 0) rho[p] = m;
}

// Forward-mode dual number: value and derivative along one direction.
struct Dual {
    double v, d;
    __device__ Dual(double x = 0.0) : v(x), d(0.0) {}
    __device__ Dual(double x, double dx) : v(x), d(dx) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.v * b.d + a.d * b.v); }
__device__ inline Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}

// The model for the screen of many sets: M (Eq. 5, M[k][i] = m_k(v_i)), its
// inverse and the velocities v[i][2], in FP64; filled once per device.
__device__ double screen_model[2 * NQ * NQ + 2 * NQ];

// Many parameter sets: matrix idx = q n + j is set q at phase pair j.  Each
// group builds its own C = dt M^-1 S (M - J M_c) from its set's state and
// rates (J, the Jacobian of Eq. 14 through rho, j, e, by dual numbers: lane c
// < 4 takes the derivative along conserved moment c), then G = diag(lw) - C.
__global__ __launch_bounds__(64) void k_screen_sets(ScreenSetArgs a)
{
    __shared__ ScreenLds L;
    __shared__ double Js[SCREEN_PER_BLOCK][NQ][4];
    const int g = threadIdx.x / SCREEN_GROUP, t = threadIdx.x % SCREEN_GROUP;
    const long long idx = (long long)blockIdx.x * SCREEN_PER_BLOCK + g;
    if (idx >= (long long)a.nsets * a.n) return;  // the whole group
    const int q = (int)(idx / a.n), j = (int)(idx % a.n);
    const double *M = screen_model, *Minv = screen_model + NQ * NQ, *vel = screen_model + 2 * NQ * NQ;
    const double rho = a.states[4 * q], ux = a.states[4 * q + 1], uy = a.states[4 * q + 2],
                 T = a.states[4 * q + 3];
    bool ok = rho > 0.0 && T > 0.0 && isfinite(rho + ux + uy + T);
    for (int k = 0; k < NQ; ++k) ok = ok && isfinite(a.rates[(long long)NQ * q + k]);
    const double tx = a.theta[2 * j], ty = a.theta[2 * j + 1];
    ok = ok && isfinite(tx) && isfinite(ty);
    if (!ok) {  // uniform over the group
        if (a.rho && t == 0) a.rho[idx] = NAN;
        if (a.max && t == 0) atomicMax((unsigned long long *)&a.max[q], (unsigned long long)__double_as_longlong(NAN));
        return;
    }
    if (t < 4) {  // column t of J = d f-hat^eq / d (rho, j_x, j_y, e)
        const Dual c0(rho, t == 0 ? 1.0 : 0.0), c1(rho * ux, t == 1 ? 1.0 : 0.0),
            c2(rho * uy, t == 2 ? 1.0 : 0.0), c3(rho * (T + 0.5 * (ux * ux + uy * uy)), t == 3 ? 1.0 : 0.0);
        Dual h[NQ];
        feq_of_conserved(c0, c1, c2, c3, h);
        for (int k = 0; k < NQ; ++k) Js[g][k][t] = h[k].d;
    }
    wave_sync();
    double D[NQ];  // column t of M - J M_c
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        double acc = M[k * NQ + t];
        for (int c = 0; c < 4; ++c) acc -= Js[g][k][c] * M[c * NQ + t];
        D[k] = acc * a.rates[(long long)NQ * q + k];
    }
    const double ax = vel[2 * t] * a.dt / a.dx, by = vel[2 * t + 1] * a.dt / a.dy;
    const double2 lw = lw_factor(ax, by, tx, ty);
    for (int r = 0; r < NQ; ++r) {  // lane t builds column t
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NQ; ++k) acc += Minv[r * NQ + k] * D[k];
        double2 e = make_double2(-a.dt * acc, 0.0);
        if (r == t) e = c_add(e, lw);
        L.A[g][r][t] = e;
    }
    wave_sync();
    double2 e;
    double m;
    int rank;
    screen_eig(L, g, t, e, m, rank);
    if (rank == 0) {
        if (a.rho) a.rho[idx] = m;
        if (a.max) atomicMax((unsigned long long *)&a.max[q], (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_fill_f64(double *p, long long n, double value)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

inline unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------------ launchers

template <class Real>
hipError_t launch_init(const Field &F, const ConstsT<Real> &K, Real *f, const float *rho,
                       const float *ux, const float *uy, const float *T, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_init<Real>), dim3(blocks_for((long long)F.nx * F.ny, 256)), dim3(256), 0,
                       s, F, K, f, rho, ux, uy, T, flag);
    return hipGetLastError();
}

template <class Real>
hipError_t launch_step_simple(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                              const Real *fin, Real *fout, const long long *d_step, int k,
                              hipStream_t s)
{
    dim3 grid(blocks_for(F.nx, 64), blocks_for(F.ny, 4));
    hipLaunchKernelGGL((k_step_simple<Real>), grid, dim3(256), 0, s, F, K, G, fin, fout, d_step, k);
    return hipGetLastError();
}

namespace {
template <int R, int AUX, class Real>
void launch_rows_variant(dim3 grid, hipStream_t s, const Field &F, const ConstsT<Real> &K,
                         const GhostsT<Real> &G, const Real *fin, Real *fout, unsigned bytes, int ncol,
                         int nrg, int nb, const long long *d_step, int k, int ord, double *slots, int fb,
                         const Bf3Ops *bops)
{
#define MRTFD_ROWS_C(Bu, Bf)                                                                       \
    hipLaunchKernelGGL((k_step_rows<R, AUX, Bu, Bf, Real>), grid, dim3(256), 0, s, F, K, G, fin,   \
                       fout, bytes, ncol, nrg, nb, d_step, k, ord, slots, Bu ? fb : 0, bops)
    if constexpr (sizeof(Real) == 4) {  // the matrix-core collision is FP32 only
        if (bops) {
            if (slots)
                MRTFD_ROWS_C(true, true);
            else
                MRTFD_ROWS_C(false, true);
            return;
        }
    }
    if (slots)
        MRTFD_ROWS_C(true, false);
    else
        MRTFD_ROWS_C(false, false);
#undef MRTFD_ROWS_C
}
}  // namespace

template <class Real>
hipError_t launch_step_rows(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                            const Real *fin, Real *fout, int rows, int stream_stores, int order,
                            const long long *d_step, int k, hipStream_t s, double *slots,
                            const Bf3Ops *bops)
{
    const int ncol = (F.nx + 63) / 64;
    const int nrg = (F.ny + rows - 1) / rows;
    const int nb = ncol * ((nrg + 3) / 4);
    const int ord = (order == 1 && (ncol & 7) == 0) ? 1 : 0;  // column bands need ncol % 8 == 0
    const long long total = (long long)sizeof(Real) * F.total;
    if (total >= (1LL << 32)) return hipErrorInvalidValue;  // buffer offsets are 32-bit
    if (sizeof(Real) == 8 && (rows != 1 || bops)) return hipErrorInvalidValue;  // FP64: one row per wave
    const unsigned bytes = (unsigned)total;
    // budget blocks: one thread per side node, rounded up to a multiple of 8
    const int fb = slots ? (int)((blocks_for(2LL * (F.nx + F.ny), 256) + 7) / 8 * 8) : 0;
    const dim3 grid(nb + fb);
    // store cache policy: 0 default, 2 non-temporal (streaming)
    if (rows == 1) {
        if (stream_stores)
            launch_rows_variant<1, 2>(grid, s, F, K, G, fin, fout, bytes, ncol, nrg, nb, d_step, k, ord,
                                      slots, fb, bops);
        else
            launch_rows_variant<1, 0>(grid, s, F, K, G, fin, fout, bytes, ncol, nrg, nb, d_step, k, ord,
                                      slots, fb, bops);
    } else if (rows == 2) {
        if constexpr (sizeof(Real) == 4) {
            if (stream_stores)
                launch_rows_variant<2, 2>(grid, s, F, K, G, fin, fout, bytes, ncol, nrg, nb, d_step, k,
                                          ord, slots, fb, bops);
            else
                launch_rows_variant<2, 0>(grid, s, F, K, G, fin, fout, bytes, ncol, nrg, nb, d_step, k,
                                          ord, slots, fb, bops);
        }
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template hipError_t launch_step_rows<float>(const Field &, const Consts &, const Ghosts &, const float *,
                                            float *, int, int, int, const long long *, int, hipStream_t,
                                            double *, const Bf3Ops *);
template hipError_t launch_step_rows<double>(const Field &, const Consts64 &, const Ghosts64 &,
                                             const double *, double *, int, int, int, const long long *,
                                             int, hipStream_t, double *, const Bf3Ops *);

hipError_t launch_fill(void *p, size_t bytes, unsigned pattern, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if ((bytes & 3) || (reinterpret_cast<uintptr_t>(p) & 15)) return hipErrorInvalidValue;
    const size_t n = bytes / 16;
    const int ntail = (int)((bytes % 16) / 4);
    const unsigned blocks = (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, static_cast<uint4 *>(p), n,
                       reinterpret_cast<unsigned *>(static_cast<char *>(p) + n * 16), ntail, pattern);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) { return launch_fill(p, bytes, 0u, s); }

hipError_t launch_counter_add(long long *d_step, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, d_step, n, 0);
    return hipGetLastError();
}

hipError_t launch_counter_set(long long *d_step, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, d_step, n, 1);
    return hipGetLastError();
}

template <class Real>
hipError_t launch_read_macro(const Field &F, const ConstsT<Real> &K, const Real *f, float *rho,
                             float *ux, float *uy, float *T, float *p, hipStream_t s)
{
    hipLaunchKernelGGL((k_read_macro<Real>), dim3(blocks_for((long long)F.nx * F.ny, 256)),
                       dim3(256), 0, s, F, K, f, rho, ux, uy, T, p);
    return hipGetLastError();
}

int sums_blocks(const Field &F)
{
    const long long n = (long long)F.nx * F.ny;
    long long b = (n + 255) / 256;
    return (int)(b < SUM_BLOCKS_MAX ? b : SUM_BLOCKS_MAX);
}

template <class Real>
hipError_t launch_sums(const Field &F, const SumW &W, const Real *f, double *partials,
                       double *out, hipStream_t s)
{
    const int nb = sums_blocks(F);
    hipLaunchKernelGGL((k_sums_partial<Real>), dim3(nb), dim3(256), 0, s, F, W, f, partials);
    hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, s, partials, nb, W, out);
    return hipGetLastError();
}

// Library-held scratch for the reduction partials of the allocation-free
// sums (4 doubles per block of k_sums_partial).  Each GPU holds its own copy
// at its own address for the life of the process; host code must use the
// address that hipGetSymbolAddress reports for the current device, never
// the symbol itself.
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch;  // device -> address of its copy of `scratch`
}  // namespace

hipError_t scratch_address(int device, double **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    double *p = nullptr;
    e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = p;
    *out = p;
    return hipSuccess;
}

template <class Real>
hipError_t launch_face_flux(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                            const FluxCoef &C, const Real *fin, double *slots,
                            const long long *d_step, int k, hipStream_t s)
{
    const long long n = 2LL * (F.nx + F.ny);
    hipLaunchKernelGGL((k_face_flux<Real>), dim3(blocks_for(n, 256)), dim3(256), 0, s, F, K, G, C,
                       fin, slots, d_step, k);
    return hipGetLastError();
}

hipError_t launch_flux_totals(int nx, int ny, const double *slots, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_flux_totals, dim3(4), dim3(256), 0, s, nx, ny, slots, out);
    return hipGetLastError();
}

template <class Src, class Dst>
hipError_t launch_pack(const Field &F, const Src *f, Dst *dst, hipStream_t s)
{
    dim3 grid(blocks_for((long long)F.nx * F.ny, 256), NQ);
    hipLaunchKernelGGL((k_pack<Src, Dst>), grid, dim3(256), 0, s, F, f, dst);
    return hipGetLastError();
}

template <class Src, class Dst>
hipError_t launch_unpack(const Field &F, const Src *src, Dst *f, hipStream_t s)
{
    dim3 grid(blocks_for((long long)F.nx * F.ny, 256), NQ);
    hipLaunchKernelGGL((k_unpack<Src, Dst>), grid, dim3(256), 0, s, F, src, f);
    return hipGetLastError();
}

// The launchers' FP32 and FP64 forms.
#define MRTFD_REAL_LAUNCHERS(Real)                                                                 \
    template hipError_t launch_init<Real>(const Field &, const ConstsT<Real> &, Real *,            \
                                          const float *, const float *, const float *,             \
                                          const float *, int *, hipStream_t);                      \
    template hipError_t launch_step_simple<Real>(const Field &, const ConstsT<Real> &,             \
                                                 const GhostsT<Real> &, const Real *, Real *,      \
                                                 const long long *, int, hipStream_t);             \
    template hipError_t launch_read_macro<Real>(const Field &, const ConstsT<Real> &, const Real *, \
                                                float *, float *, float *, float *, float *,       \
                                                hipStream_t);                                      \
    template hipError_t launch_sums<Real>(const Field &, const SumW &, const Real *, double *,     \
                                          double *, hipStream_t);                                  \
    template hipError_t launch_face_flux<Real>(const Field &, const ConstsT<Real> &,               \
                                               const GhostsT<Real> &, const FluxCoef &,            \
                                               const Real *, double *, const long long *, int,     \
                                               hipStream_t);
MRTFD_REAL_LAUNCHERS(float)
MRTFD_REAL_LAUNCHERS(double)
#undef MRTFD_REAL_LAUNCHERS
template hipError_t launch_pack<float, float>(const Field &, const float *, float *, hipStream_t);
template hipError_t launch_pack<float, double>(const Field &, const float *, double *, hipStream_t);
template hipError_t launch_pack<double, float>(const Field &, const double *, float *, hipStream_t);
template hipError_t launch_pack<double, double>(const Field &, const double *, double *, hipStream_t);
template hipError_t launch_unpack<float, float>(const Field &, const float *, float *, hipStream_t);
template hipError_t launch_unpack<float, double>(const Field &, const float *, double *, hipStream_t);
template hipError_t launch_unpack<double, float>(const Field &, const double *, float *, hipStream_t);
template hipError_t launch_unpack<double, double>(const Field &, const double *, double *, hipStream_t);

hipError_t launch_screen_sets(const ScreenSetArgs &a, hipStream_t s)
{
    const long long total = (long long)a.nsets * a.n;
    if (total <= 0) return hipSuccess;
    if (a.max) hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(a.nsets, 256)), dim3(256), 0, s, a.max, (long long)a.nsets, 0.0);
    hipLaunchKernelGGL(k_screen_sets, dim3(blocks_for(total, SCREEN_PER_BLOCK)), dim3(64), 0, s, a);
    return hipGetLastError();
}

namespace {
std::mutex g_screen_model_mu;
std::map<int, bool> g_screen_model;
}  // namespace

hipError_t screen_model_ready(int device, const double *model)
{
    std::lock_guard<std::mutex> lk(g_screen_model_mu);
    if (g_screen_model.count(device)) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    e = hipMemcpyToSymbol(HIP_SYMBOL(screen_model), model, sizeof(double) * (2 * NQ * NQ + 2 * NQ));
    if (e == hipSuccess) g_screen_model[device] = true;
    return e;
}

hipError_t launch_screen(const ScreenCoef &S, const double *theta, int n, double *eig, double *rho,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_screen, dim3(blocks_for(n, SCREEN_PER_BLOCK)), dim3(64), 0, s, S, theta, n, eig, rho);
    return hipGetLastError();
}

// ------------------------------------------------------------ tube launchers

#define MRTFD_TUBE_CONFIGS(X) X(48, 8) X(32, 16) X(56, 4)

bool tubes_config_built(int seg, int round_steps)
{
#define MRTFD_TC(Sv, Kv) if (seg == Sv && round_steps == Kv) return true;
    MRTFD_TUBE_CONFIGS(MRTFD_TC)
#undef MRTFD_TC
    return false;
}

hipError_t launch_tubes(const TubeGrid &T, const Consts *K, const TubeInfo *tubes,
                        const TubeItem *items, int nitems, int round, int seg, int round_steps,
                        const float *fin, float *fout, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
#define MRTFD_TL(Sv, Kv)                                                                           \
    if (seg == Sv && round_steps == Kv) {                                                          \
        hipLaunchKernelGGL((k_tubes<Sv, Kv>), dim3(nitems), dim3(256), 0, s, T, K, tubes, items,   \
                           round, fin, fout);                                                      \
        return hipGetLastError();                                                                  \
    }
    MRTFD_TUBE_CONFIGS(MRTFD_TL)
#undef MRTFD_TL
    return hipErrorInvalidValue;
}

hipError_t launch_tubes_init(const TubeGrid &T, const Consts &K, const TubeInfo *tubes,
                             const float *states, int ntubes, int max_n, float *f, hipStream_t s)
{
    hipLaunchKernelGGL(k_tubes_init, dim3(blocks_for(max_n, 256), ntubes), dim3(256), 0, s, T, K,
                       tubes, states, f);
    return hipGetLastError();
}

hipError_t launch_tube_macro(const TubeGrid &T, const Consts &K, const TubeInfo *tubes, int tube,
                             int n, const float *f, float *rho, float *ux, float *uy, float *Tt,
                             float *p, hipStream_t s)
{
    hipLaunchKernelGGL(k_tube_macro, dim3(blocks_for((long long)n * TUBE_ROWS, 256)), dim3(256), 0,
                       s, T, K, tubes, tube, f, rho, ux, uy, Tt, p);
    return hipGetLastError();
}

hipError_t launch_tube_pack(const TubeGrid &T, const TubeInfo *tubes, int tube, int n,
                            const float *f, float *dst, hipStream_t s)
{
    dim3 grid(blocks_for((long long)n * TUBE_ROWS, 256), NQ);
    hipLaunchKernelGGL(k_tube_pack, grid, dim3(256), 0, s, T, tubes, tube, f, dst);
    return hipGetLastError();
}

}  // namespace mrtfd
