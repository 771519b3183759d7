// lbaxi_device.hpp -- per-node arithmetic of the improved axisymmetric LB
// scheme for gfx950 (Li, He, Tang, Tao, arXiv:1003.0282), shared by the step,
// seed, macro and residual kernels of lbaxi.hip: macros, the BGK collision
// of Eqs. (12)-(13), the MRT collision of Sec. III B, the original scheme of
// Sec. II, the D2Q4 rules of Eqs. (53)-(54) and the boundary rules.
//
// Storage is deviation form: a stored f_a is f^_a - w_a rho0 and a stored h_a
// is h_a - T_ref/4 (g is stored as is).  Rounding of FP32 populations near
// w_a rho0 would otherwise eat most of the velocity signal; the arithmetic
// below is written so that only deviations are ever added to deviations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbx {

enum { SIDE_AXIS = 0, SIDE_WALL = 1, SIDE_PERIODIC = 2, SIDE_FREESLIP = 3 };
enum { SOUTH = 0, NORTH = 1, WEST = 2, EAST = 3 };
enum { F_SWIRL = 1, F_THERMAL = 2, F_MRT = 4, F_ORIG = 8, F_WETZ = 16 };
enum { MODE_PRE = 1, MODE_SPEED = 2, MODE_WETZ = 4 };

struct SideP {
  int kind, thermal, kind2, thermal2;
  double uz, ur, omega, T, r_split, omega2, T2;
};

// Everything one lattice instance needs on the device (read once per tile).
struct InstP {
  int nz, nr, cart;
  int wet;    // wall sides are wet-node walls (wall through the outer node row)
  int zou;    // with wet: radial wall nodes rebuild f by Zou-He
  int pitch;  // row stride: from a node to the node one row up (one row block)
  int c0;     // column of node i = 0 (128 bytes into a padded row)
  int plane;  // population stride: from population a to a + 1 of a node (one padded row)
  int sw, se;  // offsets of population 0's west / east ghost-column strips
  double r0;
  double tau, tau_g, tau_h;  // paper convention: nu = tau / 3
  double rho0, mu0, nu_g;
  double om0, omg0, omh0;  // 1 / (tau + 1/2) of f, g, h (om0 is the MRT s_v)
  double s_e, s_eps, s_q;  // MRT rates of the e, epsilon and q moments
  double a0, period, phase, gbeta, T_ref;
  long long off;      // element offset of the instance's populations
  long long off_fld;  // element offset of its packed [nr][nz] fields
  SideP side[4];
};

// Per-instance time level and buffer parity, for macros/residual of lattices
// that stopped stepping earlier than the rest of a batch.
struct InstDyn {
  int cur;  // 0: state in buffer A, 1: in buffer B
  int pre;  // state is pre-collision f^ (after seeding) rather than f*
  long long t;
};

// ---- D2Q9 lattice: directions (e_z, e_r) in the order
//      0 (0,0) 1 (1,0) 2 (0,1) 3 (-1,0) 4 (0,-1) 5 (1,1) 6 (-1,1) 7 (-1,-1) 8 (1,-1)
__host__ __device__ constexpr int ez9(int a) {
  return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
}
__host__ __device__ constexpr int er9(int a) {
  return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
}
__host__ __device__ constexpr double w9(int a) {
  return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp9(int a) {
  return a == 0 ? 0 : (a < 5 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5);
}
// e_r flipped: 2<->4, 5<->8, 6<->7
__host__ __device__ constexpr int mr9(int a) {
  return a == 2 ? 4 : a == 4 ? 2 : a == 5 ? 8 : a == 8 ? 5 : a == 6 ? 7 : a == 7 ? 6 : a;
}
// e_z flipped: 1<->3, 5<->6, 7<->8
__host__ __device__ constexpr int mz9(int a) {
  return a == 1 ? 3 : a == 3 ? 1 : a == 5 ? 6 : a == 6 ? 5 : a == 7 ? 8 : a == 8 ? 7 : a;
}
// ---- D2Q4: 0 (1,0) 1 (0,1) 2 (-1,0) 3 (0,-1), weights 1/4
__host__ __device__ constexpr int ez4(int a) { return a == 0 ? 1 : (a == 2 ? -1 : 0); }
__host__ __device__ constexpr int er4(int a) { return a == 1 ? 1 : (a == 3 ? -1 : 0); }
__host__ __device__ constexpr int opp4(int a) { return (a + 2) & 3; }
__host__ __device__ constexpr int mr4(int a) { return a == 1 ? 3 : (a == 3 ? 1 : a); }

// Parameters of one instance converted to the compute type, per tile.
template <typename R>
struct PR {
  R rho0, inv_rho0, mu0, tau, tau_g, tau_h, nu_g, om0, omg0, omh0, gbeta, T_ref, r0;
  R a_t;  // axial force density at the time level being processed
  R se, seps, sq, ke, gfac;  // MRT: rates, s_e / (6 s_v), 1 - s_v / 2
  int cart;
};

template <typename R>
__device__ inline PR<R> make_pr(const InstP& P, long long t) {
  PR<R> p;
  p.rho0 = (R)P.rho0;
  p.inv_rho0 = (R)(1.0 / P.rho0);
  p.mu0 = (R)P.mu0;
  p.tau = (R)P.tau;
  p.tau_g = (R)P.tau_g;
  p.tau_h = (R)P.tau_h;
  p.nu_g = (R)P.nu_g;
  p.om0 = (R)P.om0;
  p.omg0 = (R)P.omg0;
  p.omh0 = (R)P.omh0;
  p.gbeta = (R)P.gbeta;
  p.T_ref = (R)P.T_ref;
  p.r0 = (R)P.r0;
  double a = P.a0;
  if (P.period > 0.0) a = P.a0 * cos(2.0 * M_PI * (double)t / P.period + P.phase);
  p.a_t = (R)a;
  p.se = (R)P.s_e;
  p.seps = (R)P.s_eps;
  p.sq = (R)P.s_q;
  p.ke = (R)(P.s_e / (6.0 * P.om0));
  p.gfac = (R)(1.0 - 0.5 * P.om0);
  p.cart = P.cart;
  return p;
}

// Reciprocal from the hardware estimate refined by Newton steps (two for
// double, one for float): within an ulp or two of the IEEE quotient at a
// fraction of the cost of a full division sequence.
__device__ inline double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Row constants: 1/r (zero on the axis and in planar mode) and the
// direction-dependent relaxation rates omega = omega0 (1 + tau e_r / r) of
// f, g and h for e_r = +1 / -1, with the source weights 1 - omega/2 of f.
template <typename R>
struct Row {
  R ir, ir2;
  R omp, omm, c0, cp, cm;  // f (BGK)
  R gam;                   // f (MRT): gamma = (1 - s_v / 2) / r of Eqs. (47)-(50)
  R gp, gm, gsk;           // g: rates and nu_g / r
  R hp, hm;                // h
};

template <typename R, int F>
__device__ inline Row<R> make_row(const PR<R>& p, int j) {
  Row<R> w;
  const R r = p.r0 + (R)j;
  w.ir = (p.cart || !(r > (R)0)) ? (R)0 : rcp(r);
  w.ir2 = w.ir * w.ir;
  if (F & F_MRT) {
    w.gam = p.gfac * w.ir;
  } else {
    w.omp = p.om0 * ((R)1 + p.tau * w.ir);
    w.omm = p.om0 * ((R)1 - p.tau * w.ir);
    w.c0 = (R)1 - (R)0.5 * p.om0;
    w.cp = (R)1 - (R)0.5 * w.omp;
    w.cm = (R)1 - (R)0.5 * w.omm;
  }
  if (F & F_SWIRL) {
    w.gp = p.omg0 * ((R)1 + p.tau_g * w.ir);
    w.gm = p.omg0 * ((R)1 - p.tau_g * w.ir);
    w.gsk = p.nu_g * w.ir;
  }
  if (F & F_THERMAL) {
    w.hp = p.omh0 * ((R)1 + p.tau_h * w.ir);
    w.hm = p.omh0 * ((R)1 - p.tau_h * w.ir);
  }
  return w;
}

template <typename R>
struct Mac {
  R drho, rho, uz, ur, uth, dT, Fz, Fr;
};

// Eqs. (14)-(17) solved explicitly with mu -> mu0 (Sec. III A): with the
// velocity-independent force G = (a(t) + rho0 g beta (T - T_ref),
// rho0 u_th^2 / r), u_r = (sum e_r f + G_r/2) / (sum f + mu0 / r^2),
// rho = sum f / (1 + u_r / 2r), u_z = (sum e_z f + G_z/2) / sum f.
template <typename R, int F>
__device__ inline Mac<R> macros(const PR<R>& p, const Row<R>& w, bool axis_row, const R* f,
                                const R* g, const R* h) {
  Mac<R> m;
  const R ir = w.ir;
  const R s0d = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R sz = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R sr = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
  const R s0 = p.rho0 + s0d;
  R uth = (R)0;
  if ((F & F_SWIRL) && !axis_row) uth = ((g[0] + g[1]) + (g[2] + g[3])) * p.inv_rho0;
  R dT = (R)0;
  if (F & F_THERMAL) dT = (h[0] + h[1]) + (h[2] + h[3]);
  R Gz = p.a_t;
  if (F & F_THERMAL) Gz += p.rho0 * p.gbeta * dT;
  R Gr = (R)0;
  if (F & F_SWIRL) Gr = p.rho0 * uth * uth * ir;
  const R ur = (sr + (R)0.5 * Gr) * rcp(s0 + p.mu0 * w.ir2);
  const R x = (R)0.5 * ur * ir;
  m.drho = (s0d - p.rho0 * x) * rcp((R)1 + x);
  m.rho = p.rho0 + m.drho;
  m.uz = (sz + (R)0.5 * Gz) * rcp(s0);
  m.ur = ur;
  m.uth = uth;
  m.dT = dT;
  m.Fz = Gz;
  m.Fr = Gr - (R)2 * p.mu0 * ur * w.ir2;
  return m;
}

// Collision of the direction pair (a, b) with e_b = -e_a (same weight w):
// f_eq = w (drho + rho P) with P = 3 e.u + 4.5 (e.u)^2 - 1.5 u^2 (Eq. 6, in
// deviation form) and S = w (1 + P) [3 (e - u).F - rho u_r / r] (Eq. 12);
// f* = f - omega (f - f_eq) + (1 - omega/2) S (Eq. 13).
template <typename R>
__device__ inline void collide_pair(R& fa, R& fb, R eu, R eF, R w, R oma, R omb, R ca, R cb,
                                    R drho, R rho, R k15, R C0) {
  const R base = (R)4.5 * eu * eu - k15;
  const R mid = w * (drho + rho * base);
  const R odd = (R)3 * w * rho * eu;
  const R Sa = w * ((R)1 + base + (R)3 * eu) * (C0 + (R)3 * eF);
  const R Sb = w * ((R)1 + base - (R)3 * eu) * (C0 - (R)3 * eF);
  fa = fa - oma * (fa - (mid + odd)) + ca * Sa;
  fb = fb - omb * (fb - (mid - odd)) + cb * Sb;
}

// MRT collision of f (Sec. III B) with x = r, y = z.  Eq. (41) changes each
// moment of Eq. (38) by dm_k = -s_k (m_k - m_eq_k) + (1 - s_k/2) S~_k, with
// S~ = -(u_r / r) m_eq + S~' (Eq. 51); for the conserved moments this is
// S~_k exactly (f-bar = f - S/2 and the macros of Eqs. 16-17 make
// m_k - m_eq_k = -S~_k / 2), and Eqs. (49)-(50) subtract gamma [(s_e / 6 s_v)
// e1 + p_xx1 / 2] and gamma p_xy1 from the momentum rows, m1 = (m - m_eq) +
// S~/2.  The populations then change by M^-1 dm: the rows of M are
// orthogonal with squared norms (9, 36, 36, 6, 12, 6, 12, 4, 4).  Moments of
// the stored deviations d_a = f-bar_a - w_a rho0 differ from those of f-bar
// only in rho, e and epsilon (by rho0, -2 rho0, rho0), which the
// non-equilibrium parts below absorb.
template <typename R>
__device__ inline void collide_f_mrt(const PR<R>& p, const Row<R>& w, const Mac<R>& m, R* f) {
  const R ux = m.ur, uy = m.uz, Fx = m.Fr, Fy = m.Fz, rho = m.rho;
  const R u2 = ux * ux + uy * uy;
  const R uF = ux * Fx + uy * Fy;
  const R c = -ux * w.ir;  // mass-source factor -u_r / r
  // moments of the deviations: axis directions 2 (+x) 4 (-x) 1 (+y) 3 (-y),
  // diagonals 5 (+x+y) 6 (+x-y) 7 (-x-y) 8 (-x+y)
  const R A = (f[1] + f[3]) + (f[2] + f[4]);
  const R D = (f[5] + f[7]) + (f[6] + f[8]);
  const R X1 = f[2] - f[4], Y1 = f[1] - f[3];
  const R Xd = (f[5] + f[6]) - (f[7] + f[8]);
  const R Yd = (f[5] + f[8]) - (f[6] + f[7]);
  // non-equilibrium parts m_k - m_eq_k
  const R r3u2 = (R)3 * rho * u2;
  const R ne = ((R)-4 * f[0] - A + (R)2 * D) + (R)2 * m.drho - r3u2;
  const R nps = ((R)4 * f[0] - (R)2 * A + D) - m.drho + r3u2;
  const R nqx = ((R)-2 * X1 + Xd) + rho * ux;
  const R nqy = ((R)-2 * Y1 + Yd) + rho * uy;
  const R npxx = ((f[2] + f[4]) - (f[1] + f[3])) - rho * (ux * ux - uy * uy);
  const R npxy = ((f[5] + f[7]) - (f[6] + f[8])) - rho * ux * uy;
  // source moments
  const R cr = c * rho;
  const R Se = cr * ((R)-2 + (R)3 * u2) + (R)6 * uF;
  const R Sps = cr * ((R)1 - (R)3 * u2) - (R)6 * uF;
  const R Sjx = cr * ux + Fx, Sjy = cr * uy + Fy;  // S~_qx = -S~_jx, S~_qy = -S~_jy
  const R Spxx = cr * (ux * ux - uy * uy) + (R)2 * (ux * Fx - uy * Fy);
  const R Spxy = cr * ux * uy + (ux * Fy + uy * Fx);
  const R sv = p.om0;
  const R hv = (R)1 - (R)0.5 * sv;
  const R dE = -p.se * ne + ((R)1 - (R)0.5 * p.se) * Se;
  const R dP = -p.seps * nps + ((R)1 - (R)0.5 * p.seps) * Sps;
  const R hq = (R)1 - (R)0.5 * p.sq;
  const R dQx = -p.sq * nqx - hq * Sjx;
  const R dQy = -p.sq * nqy - hq * Sjy;
  const R dXX = -sv * npxx + hv * Spxx;
  const R dXY = -sv * npxy + hv * Spxy;
  const R dJx = Sjx - w.gam * (p.ke * (ne + (R)0.5 * Se) + (R)0.5 * (npxx + (R)0.5 * Spxx));
  const R dJy = Sjy - w.gam * (npxy + (R)0.5 * Spxy);
  // f += M^-1 dm
  const R r0 = cr * (R)(1.0 / 9.0);
  const R re = dE * (R)(1.0 / 36.0), rp = dP * (R)(1.0 / 36.0);
  const R jx = dJx * (R)(1.0 / 6.0), jy = dJy * (R)(1.0 / 6.0);
  const R qx = dQx * (R)(1.0 / 12.0), qy = dQy * (R)(1.0 / 12.0);
  const R px = dXX * (R)0.25, pc = dXY * (R)0.25;
  f[0] += r0 - (R)4 * re + (R)4 * rp;
  const R b1 = r0 - re - (R)2 * rp;
  const R ax = jx - (R)2 * qx, ay = jy - (R)2 * qy;
  f[2] += (b1 + px) + ax;
  f[4] += (b1 + px) - ax;
  f[1] += (b1 - px) + ay;
  f[3] += (b1 - px) - ay;
  const R b2 = r0 + (R)2 * re + rp;
  const R X = jx + qx, Y = jy + qy;
  f[5] += (b2 + pc) + (X + Y);
  f[7] += (b2 + pc) - (X + Y);
  f[6] += (b2 - pc) + (X - Y);
  f[8] += (b2 - pc) - (X - Y);
}

// ---- the original scheme (Sec. II, Eqs. 5-10) ---------------------------------
// Premnath and Abraham's scheme, kept as the comparison the paper improves
// on: constant rate omega0, source Eq. (7)
//   G_a = w_a [3 (1 + P_a)(e_a - u).F - rho u_r / r],
//   F_r = mu0 D_r / r - 2 mu0 u_r / r^2 - rho u_r^2 / r,
//   F_z = mu0 D_z / r - rho u_z u_r / r + a(t),
// macros Eqs. (9)-(10).  D_r = 2 d_r u_r and D_z = d_r u_z + d_z u_r are
// central differences of the velocity of the previous level, read from the
// lagged velocity field (lag_grad below).

// Eqs. (9)-(10) with D known: s0 = sum f = rho (1 + u_r / 2r),
// u_r = (sum e_r f + mu0 D_r / 2r) / (s0 + mu0 / r^2),
// u_z = (sum e_z f + mu0 D_z / 2r + a / 2) / s0; Fz, Fr hold Eq. (7)'s bracket.
template <typename R>
__device__ inline Mac<R> macros_orig(const PR<R>& p, const Row<R>& w, const R* f, R Dr, R Dz) {
  Mac<R> m;
  const R ir = w.ir;
  const R s0d = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R sz = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R sr = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
  const R s0 = p.rho0 + s0d;
  const R ur = (sr + (R)0.5 * p.mu0 * Dr * ir) * rcp(s0 + p.mu0 * w.ir2);
  const R x = (R)0.5 * ur * ir;
  m.drho = (s0d - p.rho0 * x) * rcp((R)1 + x);
  m.rho = p.rho0 + m.drho;
  m.uz = (sz + (R)0.5 * (p.mu0 * Dz * ir + p.a_t)) * rcp(s0);
  m.ur = ur;
  m.uth = (R)0;
  m.dT = (R)0;
  m.Fr = p.mu0 * ir * Dr - (R)2 * p.mu0 * ur * w.ir2 - m.rho * ur * ur * ir;
  m.Fz = p.mu0 * ir * Dz - m.rho * m.uz * ur * ir + p.a_t;
  return m;
}

// Eq. (8): f~ += -omega0 (f~ - f_eq) + (1 - omega0 / 2) G with G of Eq. (7),
// in deviation form (f_eq = w (drho + rho P)).
template <typename R>
__device__ inline void collide_f_orig(const PR<R>& p, const Row<R>& w, const Mac<R>& m, R* f) {
  const R uz = m.uz, ur = m.ur;
  const R k15 = (R)1.5 * (uz * uz + ur * ur);
  const R uF = uz * m.Fz + ur * m.Fr;
  const R mass = m.rho * ur * w.ir;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const R ez = (R)ez9(a), er = (R)er9(a), wa = (R)w9(a);
    const R eu = ez * uz + er * ur;
    const R Pa = (R)3 * eu + (R)4.5 * eu * eu - k15;
    const R G = wa * ((R)3 * ((R)1 + Pa) * (ez * m.Fz + er * m.Fr - uF) - mass);
    f[a] = f[a] - p.om0 * (f[a] - wa * (m.drho + m.rho * Pa)) + w.c0 * G;
  }
}

// Eq. (13) with the source of Eq. (12) for f (or the MRT collision above);
// Eq. (53)-(54) for g; the temperature analogue for h.  Updates the
// populations in place.
template <typename R, int F>
__device__ inline void collide(const PR<R>& p, const Row<R>& w, const Mac<R>& m, R* f, R* g,
                               R* h, int part = 3) {
  // part: 1 = f, 2 = g and h, 3 = all
  const R uz = m.uz, ur = m.ur;
  if (!(part & 1)) {
  } else if (F & F_MRT) {
    collide_f_mrt<R>(p, w, m, f);
  } else {
    const R k15 = (R)1.5 * (uz * uz + ur * ur);
    const R C0 = -(R)3 * (uz * m.Fz + ur * m.Fr) - m.rho * ur * w.ir;
    const R w1 = (R)(1.0 / 9.0), w5 = (R)(1.0 / 36.0);
    {
      const R w0 = (R)(4.0 / 9.0);
      const R feqd = w0 * (m.drho - m.rho * k15);
      const R S = w0 * ((R)1 - k15) * C0;
      f[0] = f[0] - p.om0 * (f[0] - feqd) + w.c0 * S;
    }
    // e = (1,0) / (-1,0); (0,1) / (0,-1); (1,1) / (-1,-1); (1,-1) / (-1,1)
    collide_pair(f[1], f[3], uz, m.Fz, w1, p.om0, p.om0, w.c0, w.c0, m.drho, m.rho, k15, C0);
    collide_pair(f[2], f[4], ur, m.Fr, w1, w.omp, w.omm, w.cp, w.cm, m.drho, m.rho, k15, C0);
    collide_pair(f[5], f[7], uz + ur, m.Fz + m.Fr, w5, w.omp, w.omm, w.cp, w.cm, m.drho, m.rho,
                 k15, C0);
    collide_pair(f[8], f[6], uz - ur, m.Fz - m.Fr, w5, w.omm, w.omp, w.cm, w.cp, m.drho, m.rho,
                 k15, C0);
  }
  if ((F & F_SWIRL) && (part & 2)) {
    // g_eq = (rho0 u_th / 4)(1 + 2 e.u), S^g = -(1/r)(2 u_r + nu / r) g_eq
    const R q = (R)0.25 * p.rho0 * m.uth;
    const R sk = (R)1 - w.ir * ((R)2 * ur + w.gsk);  // g* = g - om (g - geq) + (sk - 1) geq
    const R qz = (R)2 * q * uz, qr = (R)2 * q * ur;
    const R gz0 = q + qz, gz1 = q - qz, gr0 = q + qr, gr1 = q - qr;
    g[0] = g[0] - p.omg0 * g[0] + (p.omg0 + sk - (R)1) * gz0;
    g[2] = g[2] - p.omg0 * g[2] + (p.omg0 + sk - (R)1) * gz1;
    g[1] = g[1] - w.gp * g[1] + (w.gp + sk - (R)1) * gr0;
    g[3] = g[3] - w.gm * g[3] + (w.gm + sk - (R)1) * gr1;
  }
  if ((F & F_THERMAL) && (part & 2)) {
    // h_eq = (T/4)(1 + 2 e.u), S^h = -(u_r / r) h_eq; h stored as h - T_ref/4
    const R T = p.T_ref + m.dT;
    const R q = (R)0.25 * T, qd = (R)0.25 * m.dT;
    const R sh = -ur * w.ir;
    const R tz = (R)2 * q * uz, tr = (R)2 * q * ur;
    h[0] = h[0] - p.omh0 * (h[0] - (qd + tz)) + sh * (q + tz);
    h[2] = h[2] - p.omh0 * (h[2] - (qd - tz)) + sh * (q - tz);
    h[1] = h[1] - w.hp * (h[1] - (qd + tr)) + sh * (q + tr);
    h[3] = h[3] - w.hm * (h[3] - (qd - tr)) + sh * (q - tr);
  }
}

// ---- streaming ---------------------------------------------------------------
// Population a of node (i, j), rows j in [-1, nr] (the two ghost rows
// included), is at a * plane + (j + 1) * pitch + c0 + i, every padded row
// starting on a 128-byte boundary so that a wave's stores are aligned; the
// host lays the populations out in row blocks (plane = one padded row,
// pitch = Q of them), then per z-end one strip holding that end's ghost
// column for rows -1..nr (population a's at a * plane + sw or se).
// The step kernel pulls f_a(x) from x - e_a for every node without any test
// (the end columns then re-read from the strips what crosses a z-end); the
// ghost slots are filled after every step by the halo kernel with the
// boundary rules below, evaluated on the post-collision values of real nodes.

__device__ inline int nidx(const InstP& P, int j, int i) { return (j + 1) * P.pitch + P.c0 + i; }

// Element at byte offset boff from a population base (boff < 4 GiB: the
// host refuses lattices whose populations reach 4 GiB).
template <typename S>
__device__ inline S ldb(const S* base, unsigned boff) {
  return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename S>
__device__ inline S* ptrb(S* base, unsigned boff) {
  return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + boff);
}

// Read-only kernel inputs (tile lists, lattice parameters) go through the
// constant address space so that wave-uniform reads become scalar loads.
template <typename T>
__device__ inline T cload(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized structs only");
  typedef const __attribute__((address_space(4))) int* cptr;
  const cptr q = (cptr)p;
  // the words become the struct through a union (no type-punned pointer)
  union U {
    int w[sizeof(T) / 4];
    T v;
    __device__ U() {}
  } u;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) u.w[k] = q[k];
  return u.v;
}

// Which segment of a z-end applies at row j (second one beyond r_split).
__device__ inline void zseg(const InstP& P, const SideP& S, int j, int& kind, double& omega,
                            int& thermal, double& T) {
  if (S.r_split >= 0.0 && P.r0 + (double)j > S.r_split) {
    kind = S.kind2; omega = S.omega2; thermal = S.thermal2; T = S.T2;
  } else {
    kind = S.kind; omega = S.omega; thermal = S.thermal; T = S.T;
  }
}

// Lagged velocity at (iu, ju), at most one of them outside the lattice:
// mirrored across the axis (u_r odd) and a free-slip end (u_z odd), wrapped
// at periodic ends, 2 u_w - u beyond a halfway wall.
template <typename S, typename R>
__device__ inline void lag_end(const InstP& P, const SideP& E, const S* uz, const S* ur,
                               int iin, int iwrap, int ju, R& vz, R& vr) {
  if (E.kind == SIDE_PERIODIC) {
    vz = (R)uz[ju * P.nz + iwrap];
    vr = (R)ur[ju * P.nz + iwrap];
    return;
  }
  int kind, th;
  double om, T;
  zseg(P, E, ju, kind, om, th, T);
  const R z0 = (R)uz[ju * P.nz + iin], r0 = (R)ur[ju * P.nz + iin];
  if (kind == SIDE_FREESLIP) {
    vz = -z0;
    vr = r0;
  } else {
    vz = (R)2 * (R)E.uz - z0;
    vr = (R)2 * (R)E.ur - r0;
  }
}

template <typename S, typename R>
__device__ inline void lag_at(const InstP& P, const S* uz, const S* ur, int iu, int ju, R& vz,
                              R& vr) {
  if (iu < 0) {
    lag_end<S, R>(P, P.side[WEST], uz, ur, 0, P.nz - 1, ju, vz, vr);
  } else if (iu >= P.nz) {
    lag_end<S, R>(P, P.side[EAST], uz, ur, P.nz - 1, 0, ju, vz, vr);
  } else if (ju < 0) {
    if (P.side[SOUTH].kind == SIDE_AXIS) {
      vz = (R)uz[P.nz + iu];
      vr = -(R)ur[P.nz + iu];
    } else {
      vz = (R)2 * (R)P.side[SOUTH].uz - (R)uz[iu];
      vr = (R)2 * (R)P.side[SOUTH].ur - (R)ur[iu];
    }
  } else if (ju >= P.nr) {
    const int o = (P.nr - 1) * P.nz + iu;
    vz = (R)2 * (R)P.side[NORTH].uz - (R)uz[o];
    vr = (R)2 * (R)P.side[NORTH].ur - (R)ur[o];
  } else {
    vz = (R)uz[ju * P.nz + iu];
    vr = (R)ur[ju * P.nz + iu];
  }
}

// Gradient terms at (i, j) from the lagged field (uz, ur) of the lattice
// (packed [nr][nz]); zero where 1/r is taken as zero.
template <typename S, typename R>
__device__ inline void lag_grad(const InstP& P, const Row<R>& w, const S* uz, const S* ur, int i,
                                int j, R& Dr, R& Dz) {
  Dr = (R)0;
  Dz = (R)0;
  if (w.ir == (R)0) return;
  R zn, rn, zs, rs, ze, re, zw, rw;
  lag_at<S, R>(P, uz, ur, i, j + 1, zn, rn);
  lag_at<S, R>(P, uz, ur, i, j - 1, zs, rs);
  lag_at<S, R>(P, uz, ur, i + 1, j, ze, re);
  lag_at<S, R>(P, uz, ur, i - 1, j, zw, rw);
  Dr = rn - rs;
  Dz = (R)0.5 * (zn - zs) + (R)0.5 * (re - rw);
}

// The same for a side chosen at run time, read field by field from the
// lattice's parameter block: a whole-struct copy with a run-time choice
// between its fields would be kept in scratch memory.
__device__ inline void zseg_g(const InstP& P, const SideP* W, int j, int& kind, double& omega,
                              int& thermal, double& T) {
  const double rs = cload(&W->r_split);
  const bool second = rs >= 0.0 && P.r0 + (double)j > rs;
  kind = second ? cload(&W->kind2) : cload(&W->kind);
  omega = second ? cload(&W->omega2) : cload(&W->omega);
  thermal = second ? cload(&W->thermal2) : cload(&W->thermal);
  T = second ? cload(&W->T2) : cload(&W->T);
}

// Parameters of the z-end segment that row j of the west (or east) end
// belongs to.  Both ends' fields are read from the lattice's parameter
// block at uniform addresses (scalar loads, issued together) and the lane's
// end is then chosen value by value: no load waits on the choice.
struct ZSeg {
  int kind, thermal;
  double omega, T, uz, ur;
};

__device__ inline ZSeg zend(const InstP& P, const InstP* Pg, bool west, int j) {
  const SideP* Wp = &Pg->side[WEST];
  const SideP* Ep = &Pg->side[EAST];
  const double rsW = cload(&Wp->r_split), rsE = cload(&Ep->r_split);
  const int kW = cload(&Wp->kind), kE = cload(&Ep->kind);
  const int k2W = cload(&Wp->kind2), k2E = cload(&Ep->kind2);
  const int tW = cload(&Wp->thermal), tE = cload(&Ep->thermal);
  const int t2W = cload(&Wp->thermal2), t2E = cload(&Ep->thermal2);
  const double oW = cload(&Wp->omega), oE = cload(&Ep->omega);
  const double o2W = cload(&Wp->omega2), o2E = cload(&Ep->omega2);
  const double TW = cload(&Wp->T), TE = cload(&Ep->T);
  const double T2W = cload(&Wp->T2), T2E = cload(&Ep->T2);
  const double uzW = cload(&Wp->uz), uzE = cload(&Ep->uz);
  const double urW = cload(&Wp->ur), urE = cload(&Ep->ur);
  const double rs = west ? rsW : rsE;
  const bool second = rs >= 0.0 && P.r0 + (double)j > rs;
  ZSeg z;
  z.kind = second ? (west ? k2W : k2E) : (west ? kW : kE);
  z.thermal = second ? (west ? t2W : t2E) : (west ? tW : tE);
  z.omega = second ? (west ? o2W : o2E) : (west ? oW : oE);
  z.T = second ? (west ? T2W : T2E) : (west ? TW : TE);
  z.uz = west ? uzW : uzE;
  z.ur = west ? urW : urE;
  return z;
}

// Ghost slot (element offset from its population's base) of the upstream position (iu, ju)
// outside the lattice: beyond a z-end, the west / east strip, which holds
// the ghost column of rows -1..nr contiguously (so that filling it is a
// coalesced write, not one element per row); else the ghost row.
__device__ inline int ghost_slot(const InstP& P, int iu, int ju) {
  return iu < 0 ? P.sw + ju + 1 : (iu >= P.nz ? P.se + ju + 1 : nidx(P, ju, iu));
}

// Boundary rules: the value node (i, j) receives in direction A when its
// upstream node (i, j) - e_A lies outside the lattice.  A z-end is resolved
// before the radial sides.  s points at the instance's population 0.
//
// f: moving-wall bounce-back adds 6 w_a rho0 (e_a . u_w); the axis mirrors
// row 1; a free-slip z-end reflects e_z only.
template <typename S, int A>
__device__ inline double rule_f(const InstP& P, const InstP* Pg, const S* s, int i, int j) {
  constexpr int ez = ez9(A), er = er9(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    if (P.side[WEST].kind == SIDE_PERIODIC) {  // both ends or neither
      iu += (iu < 0) ? nz : -nz;
    } else {
      const ZSeg z = zend(P, Pg, iu < 0, j);
      if (z.kind == SIDE_FREESLIP) {
        constexpr int b = mz9(A);
        if (ju >= 0 && ju < nr) return (double)s[b * pl + nidx(P, ju, i)];
        if (ju < 0 && P.side[SOUTH].kind == SIDE_AXIS) return (double)s[mr9(b) * pl + nidx(P, 1, i)];
        return (double)s[opp9(A) * pl + nidx(P, j, i)];
      }
      return (double)s[opp9(A) * pl + nidx(P, j, i)] +
             6.0 * w9(A) * P.rho0 * (ez * z.uz + er * z.ur);
    }
  }
  if (ju < 0) {
    const SideP& W = P.side[SOUTH];
    if (W.kind == SIDE_AXIS) return (double)s[mr9(A) * pl + nidx(P, 1, iu)];  // mirror of row 1
    return (double)s[opp9(A) * pl + nidx(P, j, i)] + 6.0 * w9(A) * P.rho0 * (ez * W.uz + er * W.ur);
  }
  if (ju >= nr) {
    const SideP& W = P.side[NORTH];
    return (double)s[opp9(A) * pl + nidx(P, j, i)] + 6.0 * w9(A) * P.rho0 * (ez * W.uz + er * W.ur);
  }
  return (double)s[A * pl + nidx(P, ju, iu)];
}

// g: anti-bounce-back with rho0 u_theta,w / 2 = rho0 omega r / 2 on walls,
// zero flux on free slip; the axis value is replaced by the extrapolation.
template <typename S, int A>
__device__ inline double rule_g(const InstP& P, const InstP* Pg, const S* s, int i, int j) {
  constexpr int ez = ez4(A), er = er4(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    if (P.side[WEST].kind == SIDE_PERIODIC) {
      iu += (iu < 0) ? nz : -nz;
    } else {
      const ZSeg z = zend(P, Pg, iu < 0, j);
      if (z.kind == SIDE_FREESLIP) return (double)s[opp4(A) * pl + nidx(P, j, i)];
      return -(double)s[opp4(A) * pl + nidx(P, j, i)] + 0.5 * P.rho0 * z.omega * (P.r0 + (double)j);
    }
  }
  if (ju < 0) {
    const SideP& W = P.side[SOUTH];
    if (W.kind == SIDE_AXIS) return 0.0;
    return -(double)s[opp4(A) * pl + nidx(P, j, i)] + 0.5 * P.rho0 * W.omega * (P.r0 - 0.5);
  }
  if (ju >= nr) {
    const SideP& W = P.side[NORTH];
    return -(double)s[opp4(A) * pl + nidx(P, j, i)] +
           0.5 * P.rho0 * W.omega * (P.r0 + (double)nr - 0.5);
  }
  return (double)s[A * pl + nidx(P, ju, iu)];
}

// h (stored as h - T_ref/4): anti-bounce-back (T_w - T_ref)/2 on fixed-
// temperature walls, bounce-back on adiabatic ones, mirror on the axis.
template <typename S, int A>
__device__ inline double rule_h(const InstP& P, const InstP* Pg, const S* s, int i, int j) {
  constexpr int ez = ez4(A), er = er4(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    if (P.side[WEST].kind == SIDE_PERIODIC) {
      iu += (iu < 0) ? nz : -nz;
    } else {
      const ZSeg z = zend(P, Pg, iu < 0, j);
      if (z.kind == SIDE_WALL && z.thermal)
        return -(double)s[opp4(A) * pl + nidx(P, j, i)] + 0.5 * (z.T - P.T_ref);
      return (double)s[opp4(A) * pl + nidx(P, j, i)];
    }
  }
  if (ju < 0) {
    const SideP& W = P.side[SOUTH];
    if (W.kind == SIDE_AXIS) return (double)s[mr4(A) * pl + nidx(P, 1, iu)];
    if (W.thermal) return -(double)s[opp4(A) * pl + nidx(P, j, i)] + 0.5 * (W.T - P.T_ref);
    return (double)s[opp4(A) * pl + nidx(P, j, i)];
  }
  if (ju >= nr) {
    const SideP& W = P.side[NORTH];
    if (W.thermal) return -(double)s[opp4(A) * pl + nidx(P, j, i)] + 0.5 * (W.T - P.T_ref);
    return (double)s[opp4(A) * pl + nidx(P, j, i)];
  }
  return (double)s[A * pl + nidx(P, ju, iu)];
}

// Ghost slots that boundary node (i, j) pulls from, with their values:
// at[k] is the slot of population k (f, g, h in storage order) or -1 where the
// upstream node is a real one.
template <typename S, int F, int A>
__device__ inline void halo_gather(const InstP& P, const InstP* Pg, const S* s, int i, int j,
                                   S* v, int* at) {
  const int pl = P.plane;
  {
    const int iu = i - ez9(A), ju = j - er9(A);
    const bool out = iu < 0 || iu >= P.nz || ju < 0 || ju >= P.nr;
    at[A] = out ? A * pl + ghost_slot(P, iu, ju) : -1;
    if (out) v[A] = (S)rule_f<S, A>(P, Pg, s, i, j);
  }
  if constexpr (A < 4) {
    const int iu = i - ez4(A), ju = j - er4(A);
    const bool out = iu < 0 || iu >= P.nz || ju < 0 || ju >= P.nr;
    if (F & F_SWIRL) {
      at[9 + A] = out ? (9 + A) * pl + ghost_slot(P, iu, ju) : -1;
      if (out) v[9 + A] = (S)rule_g<S, A>(P, Pg, s + 9 * pl, i, j);
    }
    if (F & F_THERMAL) {
      constexpr int hb = (F & F_SWIRL) ? 13 : 9;
      at[hb + A] = out ? (hb + A) * pl + ghost_slot(P, iu, ju) : -1;
      if (out) v[hb + A] = (S)rule_h<S, A>(P, Pg, s + hb * pl, i, j);
    }
  }
  if constexpr (A + 1 < 9) halo_gather<S, F, A + 1>(P, Pg, s, i, j, v, at);
}

// Fill, for boundary node (i, j), every ghost slot it pulls from.  Sources
// are always real nodes and targets ghost slots, so every value is read
// before the first write: the loads of a node stay in flight together
// instead of waiting one by one behind stores to the same buffer.
template <typename S, int F>
__device__ inline void halo_fill(const InstP& P, const InstP* Pg, S* s, int i, int j) {
  constexpr int NQ = 9 + ((F & F_SWIRL) ? 4 : 0) + ((F & F_THERMAL) ? 4 : 0);
  S v[NQ];
  int at[NQ];
  halo_gather<S, F, 0>(P, Pg, s, i, j, v, at);
#pragma unroll
  for (int k = 0; k < NQ; ++k)
    if (at[k] >= 0) s[at[k]] = v[k];
}

// Populations that node (WEST ? 0 : nz - 1, j) receives across its z-end,
// from the ghost-column strip of that end (rows j - e_r, slot row + 1).
template <typename S, typename R, int F, bool WEST_END>
__device__ inline void zend_pull(const InstP& P, const S* __restrict__ s, int j, R* f, R* g, R* h) {
  const int pl = P.plane;
  constexpr int dir = WEST_END ? 1 : -1;  // e_z of the populations that cross it
  const unsigned b = (unsigned)((WEST_END ? P.sw : P.se) + j + 1);
  constexpr unsigned es = sizeof(S);
#pragma unroll
  for (int a = 0; a < 9; ++a)
    if (ez9(a) == dir) f[a] = (R)ldb(s + a * pl, (b - er9(a)) * es);
#pragma unroll
  for (int a = 0; a < 4; ++a)
    if (ez4(a) == dir) {
      if (F & F_SWIRL) g[a] = (R)ldb(s + (9 + a) * pl, (b - er4(a)) * es);
      if (F & F_THERMAL) h[a] = (R)ldb(s + (((F & F_SWIRL) ? 13 : 9) + a) * pl, (b - er4(a)) * es);
    }
}

// Populations arriving at node (i, j): a plain pull through the padded
// rows; an end column takes what crosses its z-end from that end's strip.
// pre: the buffer holds f^ itself (right after seeding), so the node reads
// its own slots.
template <typename S, typename R, int F>
__device__ inline void load_node(const InstP& P, const S* __restrict__ s, int i, int j, bool pre,
                                 R* f, R* g, R* h) {
  // Loads are written as a wave-uniform population base plus a 32-bit byte offset
  // so that they use scalar-base addressing (one offset register per row).
  const int pl = P.plane, pt = P.pitch;
  const unsigned o = (unsigned)nidx(P, j, i);
  const S* sg = s + 9 * pl;
  const S* sh = s + ((F & F_SWIRL) ? 13 : 9) * pl;
  constexpr unsigned es = sizeof(S);
  if (pre) {
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = (R)ldb(s + a * pl, o * es);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (F & F_SWIRL) g[a] = (R)ldb(sg + a * pl, o * es);
      if (F & F_THERMAL) h[a] = (R)ldb(sh + a * pl, o * es);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = (R)ldb(s + a * pl, (o - er9(a) * pt - ez9(a)) * es);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const unsigned q = (o - er4(a) * pt - ez4(a)) * es;
      if (F & F_SWIRL) g[a] = (R)ldb(sg + a * pl, q);
      if (F & F_THERMAL) h[a] = (R)ldb(sh + a * pl, q);
    }
    // an end column takes what crosses its z-end from that end's strip
    // (re-read after the plain pull, which keeps the interior's immediate
    // load offsets and registers as they are)
    if (i == 0) zend_pull<S, R, F, true>(P, s, j, f, g, h);
    if (i == P.nz - 1) zend_pull<S, R, F, false>(P, s, j, f, g, h);
  }
}

}  // namespace lbx
