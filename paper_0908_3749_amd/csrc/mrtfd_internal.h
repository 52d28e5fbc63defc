// Internal declarations shared by the host side (mrtfd_host.cpp) and the
// kernels (mrtfd_kernels.hip) of the MRT finite-difference lattice Boltzmann
// library.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mrtfd {

constexpr int NQ = 16;

// Constants of one step (FP32, or FP64 in the FP64 mode).  The moment
// transform f-hat = M f is done in two
// stages.  Stage 1, a butterfly of adds per velocity group g (4 velocities
// each): A_g = sum of the group, X_g / Y_g = the combinations odd in v_x /
// v_y, Q_g = the quadrupole combination.  Stage 2, small dense blocks that
// mix the groups: every row of M is a radial weight times one angular
// harmonic (Sect. III.A builds M from SO(2) irreducible representations), so
// M = B P with P the butterfly and B block diagonal:
//   harmonic 0 (m1, m4, m11, m12) <- A_0..3, cos (m2, m7, m9, m15) <- X_0..3,
//   sin (m3, m8, m10, m16) <- Y_0..3, axis quadrupole (m5, m13) <- Q_0, Q_1,
//   diagonal quadrupole (m6, m14) <- Q_2, Q_3.
// The inverse is P^-1 B^-1 with the butterfly's 1/4 and 1/2 scales folded
// into the rows of B^-1, so that the inverse butterfly is adds only.
template <class Real>
struct ConstsT {
    Real f0[4][4];   // rows m1, m4, m11, m12; columns A0..A3
    Real fx[4][4];   // rows m2, m7, m9, m15;  columns X0..X3
    Real fy[4][4];   // rows m3, m8, m10, m16; columns Y0..Y3
    Real fqa[2][2];  // rows m5, m13; columns Q0, Q1
    Real fqd[2][2];  // rows m6, m14; columns Q2, Q3
    Real i0[4][4];   // rows A'0..3; columns m1, m4, m11, m12 (scaled)
    Real ix[4][4];   // rows X'0..3; columns m2, m7, m9, m15
    Real iy[4][4];   // rows Y'0..3; columns m3, m8, m10, m16
    Real iqa[2][2];  // rows Q'0, Q'1; columns m5, m13
    Real iqd[2][2];  // rows Q'2, Q'3; columns m6, m14
    // collision back-map: inverse blocks times dt*s_k (nonconserved columns)
    Real c0[4][2];   // columns m11, m12
    Real cx[4][3];   // columns m7, m9, m15
    Real cy[4][3];   // columns m8, m10, m16
    Real cqa[2][2];  // columns m5, m13
    Real cqd[2][2];  // columns m6, m14
    // Lax-Wendroff + Euler weights per population: f + cE (fE - f) + cW (fW - f)
    // + cN (fN - f) + cS (fS - f), cE = (a^2 - a)/2, cW = (a^2 + a)/2 with
    // a = v_x dt / dx (likewise N/S with b = v_y dt / dy).
    Real lw[NQ][4];  // cE, cW, cN, cS
    // Reference state at rest: the copies of f hold g = f - f^eq(rho0, 0, 0,
    // T0); e0 = rho0 T0 is its energy and Te0 = T0 e0.  All zero when no
    // reference is set (g = f).
    Real rho0, T0, e0, Te0;
};
using Consts = ConstsT<float>;
using Consts64 = ConstsT<double>;

// Device layout of one copy of f (FP32 values, FP64 in the FP64 mode: the
// same element offsets).  Rows j = -1 .. ny of 16 x `pitch` elements;
// column i sits at c = xoff + i (xoff = 64 keeps every interior row start
// 256-byte aligned; the ring around the interior is padding that no kernel
// reads), and node (i, j) of population q at
//   q * qstride + (j + 1) * jstride + (c / 64) * tstride + c % 64.
// Three orders: population planes (qstride = (ny + 2) pitch, jstride =
// pitch, tstride = 64), rows of interleaved populations (qstride = pitch,
// jstride = 16 pitch, tstride = 64: the 16 populations of a row lie next to
// each other), and tiles (qstride = 64, jstride = 16 pitch, tstride = 1024:
// each 64-column piece of a row holds its 16 populations in 4 KiB).
struct Field {
    int nx, ny;
    int pitch, xoff;
    long long qstride, jstride, tstride;
    long long total;  // elements in one copy
    __host__ __device__ long long col(int i) const {
        const int c = xoff + i;
        return (long long)(c >> 6) * tstride + (c & 63);
    }
    __host__ __device__ long long at(int q, int i, int j) const {
        return (long long)q * qstride + (long long)(j + 1) * jstride + col(i);
    }
};

// BF16 operands of the factored transform's eight 4x4 blocks for the
// matrix instruction v_mfma_f32_4x4x4_16b_bf16, where lane l supplies row
// l % 4; w[b][i] = row i of block b, two BF16 values per 32-bit word,
// element 0 low.  Forward blocks: 0 f0, 1 fx, 2 fy (columns A/X/Y 0..3; the
// diagonal groups' columns 2, 3 of fx and fy divided by sqrt 2), 3 the
// quadrupole block (rows m5, m13, m6, m14 over Q0..Q3): every entry exact in
// BF16, held in (.x, .y).  Back-map blocks: 4 c0 (columns m11, m12, 0, 0),
// 5 cx (m7, m9, m15, 0), 6 cy (m8, m10, m16, 0), 7 the quadrupole back-map
// (rows Q0..Q3 over m5, m13, m6, m14), with dt s_k folded in as in Consts:
// each FP32 entry split exactly into three BF16 parts, the high parts in
// (.x, .y) and the middle ones in (.z, .w) of w[b], the low ones in (.x,
// .y) of w[b + 4].
struct Bf3Ops {
    uint4 w[12][4];
};

enum Kind { K_PERIODIC = 0, K_DIRICHLET = 1, K_REFLECT = 2, K_EXTRAPOLATE = 3, K_WALL = 4 };

template <class Real>
struct GhostSideT {
    int kind_lo, kind_hi;
    Real st_lo[4], st_hi[4];        // rho - rho0, u1, u2, T - T0 (host FP64, rounded)
    Real feq_lo[NQ], feq_hi[NQ];    // f^eq - f_ref of the states (host FP64, rounded)
    double split0, split_rate;      // rule switch point along the side
    double h;                       // node spacing along the side
};

struct FluxCoef;

template <class Real>
struct GhostsT {
    GhostSideT<Real> side[4];  // west, east, south, north
    double dt;
    int per_x, per_y;   // periodic in x (west/east) / in y (south/north)
    // device copies of the step constants and of this struct: the boundary
    // paths of the step kernels read these, so that the interior path keeps
    // the kernel arguments to itself
    const ConstsT<Real> *kd;
    const GhostsT<Real> *gd;
    const FluxCoef *fd;  // device copy of the outflow-budget coefficients
};
using GhostSide = GhostSideT<float>;
using Ghosts = GhostsT<float>;
using Ghosts64 = GhostsT<double>;

// Launchers (mrtfd_kernels.hip).  All enqueue on `s` and return the HIP
// status of the launch.  Those templated on Real exist for float (FP32
// storage) and double (the FP64 mode).
template <class Real>
hipError_t launch_init(const Field &F, const ConstsT<Real> &K, Real *f, const float *rho,
                       const float *ux, const float *uy, const float *T, int *flag,
                       hipStream_t s);
// One time step from fin to fout at step index *d_step + k (the boundary
// rules read the clock from there).
template <class Real>
hipError_t launch_step_simple(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                              const Real *fin, Real *fout, const long long *d_step, int k,
                              hipStream_t s);
// rows per wave (1 or 2); stream_stores: non-temporal stores; order: tiles
// to XCDs in bands of tile rows (0) or of tile columns (1, when the number of
// tile columns divides by 8; else 0).  slots != nullptr: the launch also
// adds the step's outflow budget (as launch_face_flux) in leading blocks of
// its own grid (constants from the device copies G.kd, G.gd, G.fd).
// bops != nullptr (device copy of the block table): the collision's
// transforms in split-BF16 on the matrix cores.
// In FP64 (Real = double) one row per wave and no matrix-core collision.
template <class Real>
hipError_t launch_step_rows(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                            const Real *fin, Real *fout, int rows, int stream_stores, int order,
                            const long long *d_step, int k, hipStream_t s,
                            double *slots = nullptr, const Bf3Ops *bops = nullptr);
// Outflow budget (FP64).  cx[q] = {(dt/dx) v_qx / 2, (dt/dx) v_qx^2 dt / (2 dx)}
// and likewise cy along y: the face value of the A.1b difference between a
// node at the lower coordinate (lo) and the next one (hi) is
// cx[q][0] (lo + hi) - cx[q][1] (hi - lo).  w[k][q] = m_{k+1}(v_q), k < 4.
struct FluxCoef {
    double cx[NQ][2], cy[NQ][2];
    double w[4][NQ];
};
// Per step: add each side node's outflow of (rho, j1, j2, e) to its slot
// (slots: 4 doubles per node, west rows, east rows, south columns, north
// columns).  Then, on demand, the per-side totals into out[16].
template <class Real>
hipError_t launch_face_flux(const Field &F, const ConstsT<Real> &K, const GhostsT<Real> &G,
                            const FluxCoef &C, const Real *fin, double *slots,
                            const long long *d_step, int k, hipStream_t s);
hipError_t launch_flux_totals(int nx, int ny, const double *slots, double *out, hipStream_t s);

// Fill `bytes` (a multiple of 4) at p (16-byte aligned) with a 32-bit pattern,
// or with zeros, by a kernel, not a memset node.
hipError_t launch_fill(void *p, size_t bytes, unsigned pattern, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_counter_add(long long *d_step, long long n, hipStream_t s);
hipError_t launch_counter_set(long long *d_step, long long n, hipStream_t s);
template <class Real>
hipError_t launch_read_macro(const Field &F, const ConstsT<Real> &K, const Real *f, float *rho,
                             float *ux, float *uy, float *T, float *p, hipStream_t s);
// FP64 weights of the conserved rows m1..m4 at the 16 velocities, and the
// reference state's share of the totals (its moments times the node count),
// added once at the end.
struct SumW {
    double w[4][NQ];
    double add[4];
};
// At most SUM_BLOCKS_MAX blocks of 4 partial sums each.
constexpr int SUM_BLOCKS_MAX = 1024;
constexpr int SCRATCH_DOUBLES = 4 * SUM_BLOCKS_MAX;
int sums_blocks(const Field &F);
// partials: 4 * sums_blocks(F) doubles; out: 4 doubles (device).
template <class Real>
hipError_t launch_sums(const Field &F, const SumW &W, const Real *f, double *partials,
                       double *out, hipStream_t s);
// Device address of the library's file-scope scratch array (SCRATCH_DOUBLES
// doubles) on `device`, which must be the current device: looked up with
// hipGetSymbolAddress on the first call per device and kept.
hipError_t scratch_address(int device, double **out);
// Stored values between a copy of f and a packed [16][ny][nx] array of the
// same or the other precision (Src -> Dst, rounded to nearest where narrower).
template <class Src, class Dst>
hipError_t launch_pack(const Field &F, const Src *f, Dst *dst, hipStream_t s);
template <class Src, class Dst>
hipError_t launch_unpack(const Field &F, const Src *src, Dst *f, hipStream_t s);

// Von Neumann screen (Sect. IV): the amplification matrix of one Fourier
// mode around a uniform state is G(theta) = diag(adv_i(theta)) - C with
// adv_i = 1 - i a_i sin(theta_x) + a_i^2 (cos(theta_x) - 1) - i b_i
// sin(theta_y) + b_i^2 (cos(theta_y) - 1), a_i = v_ix dt / dx, b_i = v_iy dt
// / dy (Eq. A.1b), and C = dt M^-1 S (M - d f-hat^eq / d f), the same for
// every phase.
struct ScreenCoef {
    double C[NQ][NQ];
    double a[NQ], b[NQ];
};
// f-hat^eq of Eq. (14) as a function of the conserved moments (rho, j_x, j_y,
// e), with P = e - |j|^2 / (2 rho); generic in the number type, so that its
// Jacobian can be taken by complex steps.
template <class Num>
__host__ __device__ inline void feq_of_conserved(Num rho, Num jx, Num jy, Num e, Num (&h)[NQ])
{
    const Num r = Num(1.0) / rho;
    const Num j2 = jx * jx + jy * jy;
    const Num P = e - Num(0.5) * j2 * r;
    const Num g = Num(6.0) * rho * e - Num(2.0) * j2;
    h[0] = rho;
    h[1] = jx;
    h[2] = jy;
    h[3] = e;
    h[4] = (jx * jx - jy * jy) * r;
    h[5] = jx * jy * r;
    h[6] = (e + P) * jx * r;
    h[7] = (e + P) * jy * r;
    h[8] = (jx * jx - Num(3.0) * jy * jy) * jx * r * r;
    h[9] = (Num(3.0) * jx * jx - jy * jy) * jy * r * r;
    h[10] = Num(2.0) * e * e * r - Num(0.25) * j2 * j2 * r * r * r;
    h[11] = Num(0.0);
    h[12] = g * (jx * jx - jy * jy) * r * r * r;
    h[13] = g * jx * jy * r * r * r;
    h[14] = Num(0.0);
    h[15] = Num(0.0);
}

// Many parameter sets at once (mrtfd_screen_sets): set q has the state
// states[4 q ..] = (rho, u1, u2, T) and the rates rates[16 q ..]; matrix q n
// + j is set q at phase pair theta[2 j], theta[2 j + 1] (device arrays).
// Writes max |omega| to rho[q n + j] and the largest over j to max[q] (either
// may be null; max must hold 0 beforehand), NaN for an invalid set or phase.
struct ScreenSetArgs {
    const double *states, *rates, *theta;
    double *rho, *max;
    int nsets, n;
    double dx, dy, dt;
};
hipError_t launch_screen_sets(const ScreenSetArgs &a, hipStream_t s);
// Uploads M, M^-1 and the velocities (2 * 256 + 32 doubles) for the screen
// of many sets to the current device, once per device.
hipError_t screen_model_ready(int device, const double *model);

// For each of n phase pairs theta[2 p], theta[2 p + 1] (device array): the
// 16 eigenvalues of G, largest modulus first, as (re, im) pairs at eig[32 p
// ..] and their largest modulus at rho[p] (either pointer may be null); NaN
// where the QR iteration does not converge.
hipError_t launch_screen(const ScreenCoef &S, const double *theta, int n, double *eig, double *rho,
                         hipStream_t s);

// ------------------------------------------------------------------ tubes
// Batched independent tubes: tube k has n columns and TUBE_ROWS rows,
// periodic in y, f = f^eq of its left / right state beyond its two ends.  All
// tubes live side by side in one FP32 array per copy: population q, row y,
// column x of tube k at q * plane + y * ncols + start + x, ncols = sum of n.
constexpr int TUBE_ROWS = 4;

struct TubeInfo {
    int n, start, steps, pad;
    float feq_left[NQ], feq_right[NQ];
};

struct TubeItem {  // one work item: columns [x0, x0 + seg) of a tube
    int tube, x0;
};

struct TubeGrid {
    long long plane;  // TUBE_ROWS * ncols
    int ncols;
};

// One round: every listed item advances min(round_steps, steps - round *
// round_steps) steps.  seg/round_steps must be one of the built pairs; K is a
// device copy of the constants.
hipError_t launch_tubes(const TubeGrid &T, const Consts *K, const TubeInfo *tubes,
                        const TubeItem *items, int nitems, int round, int seg, int round_steps,
                        const float *fin, float *fout, hipStream_t s);
bool tubes_config_built(int seg, int round_steps);
// f = f^eq of the left state for x < n/2 and of the right state beyond, per
// tube; states = device [ntubes][2][4] (rho, u1, u2, T).
hipError_t launch_tubes_init(const TubeGrid &T, const Consts &K, const TubeInfo *tubes,
                             const float *states, int ntubes, int max_n, float *f, hipStream_t s);
hipError_t launch_tube_macro(const TubeGrid &T, const Consts &K, const TubeInfo *tubes, int tube,
                             int n, const float *f, float *rho, float *ux, float *uy, float *Tt,
                             float *p, hipStream_t s);
hipError_t launch_tube_pack(const TubeGrid &T, const TubeInfo *tubes, int tube, int n,
                            const float *f, float *dst, hipStream_t s);

}  // namespace mrtfd
