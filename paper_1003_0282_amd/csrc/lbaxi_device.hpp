// lbaxi_device.hpp -- per-node arithmetic of the improved axisymmetric LB
// scheme for gfx950 (Li, He, Tang, Tao, arXiv:1003.0282), shared by the step,
// seed, macro and residual kernels of lbaxi.hip.
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
enum { F_SWIRL = 1, F_THERMAL = 2 };
enum { MODE_PRE = 1, MODE_SPEED = 2 };

struct SideP {
  int kind, thermal, kind2, thermal2;
  double uz, ur, omega, T, r_split, omega2, T2;
};

// Everything one lattice instance needs on the device (read once per tile).
struct InstP {
  int nz, nr, plane, cart;
  double r0;
  double tau, tau_g, tau_h;  // paper convention: nu = tau / 3
  double rho0, mu0, nu_g;
  double om0, omg0, omh0;  // 1 / (tau + 1/2) of f, g, h
  double a0, period, phase, gbeta, T_ref;
  long long off;      // element offset of the instance's population planes
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
  R rho0, mu0, tau, tau_g, tau_h, nu_g, om0, omg0, omh0, gbeta, T_ref, r0;
  R a_t;  // axial force density at the time level being processed
  int cart;
};

template <typename R>
__device__ inline PR<R> make_pr(const InstP& P, long long t) {
  PR<R> p;
  p.rho0 = (R)P.rho0;
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
  p.cart = P.cart;
  return p;
}

// 1/r of row j; every 1/r term vanishes on the axis and in planar mode.
template <typename R>
__device__ inline R inv_radius(const PR<R>& p, int j) {
  R r = p.r0 + (R)j;
  return (p.cart || !(r > (R)0)) ? (R)0 : (R)1 / r;
}

template <typename R>
struct Mac {
  R drho, rho, uz, ur, uth, dT, Fz, Fr, ir;
};

// Eqs. (14)-(17) solved explicitly with mu -> mu0 (Sec. III A): with the
// velocity-independent force G = (a(t) + rho0 g beta (T - T_ref),
// rho0 u_th^2 / r), u_r = (sum e_r f + G_r/2) / (sum f + mu0 / r^2),
// rho = sum f / (1 + u_r / 2r), u_z = (sum e_z f + G_z/2) / sum f.
template <typename R, int F>
__device__ inline Mac<R> macros(const PR<R>& p, int j, bool axis_row, const R* f, const R* g,
                                const R* h) {
  Mac<R> m;
  const R ir = inv_radius(p, j);
  const R s0d = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R sz = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R sr = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
  const R s0 = p.rho0 + s0d;
  R uth = (R)0;
  if ((F & F_SWIRL) && !axis_row) uth = ((g[0] + g[1]) + (g[2] + g[3])) / p.rho0;
  R dT = (R)0;
  if (F & F_THERMAL) dT = (h[0] + h[1]) + (h[2] + h[3]);
  R Gz = p.a_t;
  if (F & F_THERMAL) Gz += p.rho0 * p.gbeta * dT;
  R Gr = (R)0;
  if (F & F_SWIRL) Gr = p.rho0 * uth * uth * ir;
  const R ur = (sr + (R)0.5 * Gr) / (s0 + p.mu0 * ir * ir);
  const R x = (R)0.5 * ur * ir;
  m.drho = (s0d - p.rho0 * x) / ((R)1 + x);
  m.rho = p.rho0 + m.drho;
  m.uz = (sz + (R)0.5 * Gz) / s0;
  m.ur = ur;
  m.uth = uth;
  m.dT = dT;
  m.Fz = Gz;
  m.Fr = Gr - (R)2 * p.mu0 * ur * ir * ir;
  m.ir = ir;
  return m;
}

// Eq. (13) with the source of Eq. (12) for f; Eq. (53)-(54) for g; the
// temperature analogue for h.  Updates the populations in place.
template <typename R, int F>
__device__ inline void collide(const PR<R>& p, const Mac<R>& m, R* f, R* g, R* h) {
  const R uz = m.uz, ur = m.ur, ir = m.ir;
  const R usq = uz * uz + ur * ur;
  const R omp = p.om0 * ((R)1 + p.tau * ir);
  const R omm = p.om0 * ((R)1 - p.tau * ir);
  const R rur = m.rho * ur * ir;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const R ez = (R)ez9(a), er = (R)er9(a), w = (R)w9(a);
    const R eu = ez * uz + er * ur;
    const R P = (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * usq;
    const R feqd = w * (m.drho + m.rho * P);
    const R S = w * ((R)1 + P) * ((R)3 * ((ez - uz) * m.Fz + (er - ur) * m.Fr) - rur);
    const R om = er9(a) > 0 ? omp : (er9(a) < 0 ? omm : p.om0);
    f[a] = f[a] - om * (f[a] - feqd) + ((R)1 - (R)0.5 * om) * S;
  }
  if (F & F_SWIRL) {
    const R gp = p.omg0 * ((R)1 + p.tau_g * ir);
    const R gm = p.omg0 * ((R)1 - p.tau_g * ir);
    const R q = (R)0.25 * p.rho0 * m.uth;
    const R sk = -ir * ((R)2 * ur + p.nu_g * ir);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const R eu = (R)ez4(a) * uz + (R)er4(a) * ur;
      const R geq = q * ((R)1 + (R)2 * eu);
      const R om = er4(a) > 0 ? gp : (er4(a) < 0 ? gm : p.omg0);
      g[a] = g[a] - om * (g[a] - geq) + sk * geq;
    }
  }
  if (F & F_THERMAL) {
    const R hp = p.omh0 * ((R)1 + p.tau_h * ir);
    const R hm = p.omh0 * ((R)1 - p.tau_h * ir);
    const R T = p.T_ref + m.dT;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const R eu = (R)ez4(a) * uz + (R)er4(a) * ur;
      const R heq = (R)0.25 * T * ((R)1 + (R)2 * eu);
      const R heqd = (R)0.25 * (m.dT + T * (R)2 * eu);
      const R om = er4(a) > 0 ? hp : (er4(a) < 0 ? hm : p.omh0);
      h[a] = h[a] - om * (h[a] - heqd) - ur * ir * heq;
    }
  }
}

// ---- streaming: pull from the post-collision buffer ------------------------
// s points at the instance's first plane; planes are nr*nz elements, z fastest.

// Which segment of a z-end applies at row j (second one beyond r_split).
__device__ inline void zseg(const InstP& P, const SideP& S, int j, int& kind, double& omega,
                            int& thermal, double& T) {
  if (S.r_split >= 0.0 && P.r0 + (double)j > S.r_split) {
    kind = S.kind2; omega = S.omega2; thermal = S.thermal2; T = S.T2;
  } else {
    kind = S.kind; omega = S.omega; thermal = S.thermal; T = S.T;
  }
}

template <typename R, int A>
__device__ inline R pull_f_edge(const InstP& P, const R* s, int i, int j) {
  constexpr int ez = ez9(A), er = er9(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    const SideP& S = P.side[iu < 0 ? WEST : EAST];
    if (S.kind == SIDE_PERIODIC) {
      iu += (iu < 0) ? nz : -nz;
    } else {
      int kind, th; double om, T;
      zseg(P, S, j, kind, om, th, T);
      if (kind == SIDE_FREESLIP) {
        constexpr int b = mz9(A);
        if (ju >= 0 && ju < nr) return s[b * pl + ju * nz + i];
        if (ju < 0 && P.side[SOUTH].kind == SIDE_AXIS) return s[mr9(b) * pl + nz + i];
        return s[opp9(A) * pl + j * nz + i];
      }
      return s[opp9(A) * pl + j * nz + i] +
             (R)(6.0 * w9(A) * P.rho0 * (ez * S.uz + er * S.ur));
    }
  }
  if (ju < 0) {
    const SideP& S = P.side[SOUTH];
    if (S.kind == SIDE_AXIS) return s[mr9(A) * pl + nz + iu];  // mirror of row 1
    return s[opp9(A) * pl + j * nz + i] + (R)(6.0 * w9(A) * P.rho0 * (ez * S.uz + er * S.ur));
  }
  if (ju >= nr) {
    const SideP& S = P.side[NORTH];
    return s[opp9(A) * pl + j * nz + i] + (R)(6.0 * w9(A) * P.rho0 * (ez * S.uz + er * S.ur));
  }
  return s[A * pl + ju * nz + iu];
}

template <typename R, int A>
__device__ inline R pull_g_edge(const InstP& P, const R* s, int i, int j) {
  constexpr int ez = ez4(A), er = er4(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    const SideP& S = P.side[iu < 0 ? WEST : EAST];
    if (S.kind == SIDE_PERIODIC) {
      iu += (iu < 0) ? nz : -nz;
    } else {
      int kind, th; double om, T;
      zseg(P, S, j, kind, om, th, T);
      if (kind == SIDE_FREESLIP) return s[opp4(A) * pl + j * nz + i];
      return -s[opp4(A) * pl + j * nz + i] + (R)(0.5 * P.rho0 * om * (P.r0 + (double)j));
    }
  }
  if (ju < 0) {
    const SideP& S = P.side[SOUTH];
    if (S.kind == SIDE_AXIS) return (R)0;  // replaced by the axis extrapolation
    return -s[opp4(A) * pl + j * nz + i] + (R)(0.5 * P.rho0 * S.omega * (P.r0 - 0.5));
  }
  if (ju >= nr) {
    const SideP& S = P.side[NORTH];
    return -s[opp4(A) * pl + j * nz + i] +
           (R)(0.5 * P.rho0 * S.omega * (P.r0 + (double)nr - 0.5));
  }
  return s[A * pl + ju * nz + iu];
}

template <typename R, int A>
__device__ inline R pull_h_edge(const InstP& P, const R* s, int i, int j) {
  constexpr int ez = ez4(A), er = er4(A);
  const int nz = P.nz, nr = P.nr, pl = P.plane;
  int iu = i - ez;
  const int ju = j - er;
  if (iu < 0 || iu >= nz) {
    const SideP& S = P.side[iu < 0 ? WEST : EAST];
    if (S.kind == SIDE_PERIODIC) {
      iu += (iu < 0) ? nz : -nz;
    } else {
      int kind, th; double om, T;
      zseg(P, S, j, kind, om, th, T);
      if (kind == SIDE_WALL && th) return -s[opp4(A) * pl + j * nz + i] + (R)(0.5 * (T - P.T_ref));
      return s[opp4(A) * pl + j * nz + i];
    }
  }
  if (ju < 0) {
    const SideP& S = P.side[SOUTH];
    if (S.kind == SIDE_AXIS) return s[mr4(A) * pl + nz + iu];
    if (S.thermal) return -s[opp4(A) * pl + j * nz + i] + (R)(0.5 * (S.T - P.T_ref));
    return s[opp4(A) * pl + j * nz + i];
  }
  if (ju >= nr) {
    const SideP& S = P.side[NORTH];
    if (S.thermal) return -s[opp4(A) * pl + j * nz + i] + (R)(0.5 * (S.T - P.T_ref));
    return s[opp4(A) * pl + j * nz + i];
  }
  return s[A * pl + ju * nz + iu];
}

template <typename R, int F, int A>
struct EdgeLoader {
  __device__ static inline void run(const InstP& P, const R* s, int i, int j, R* f, R* g, R* h) {
    f[A] = pull_f_edge<R, A>(P, s, i, j);
    if constexpr (A < 4) {
      if (F & F_SWIRL) g[A] = pull_g_edge<R, A>(P, s + 9 * P.plane, i, j);
      if (F & F_THERMAL)
        h[A] = pull_h_edge<R, A>(P, s + ((F & F_SWIRL) ? 13 : 9) * P.plane, i, j);
    }
    if constexpr (A + 1 < 9) EdgeLoader<R, F, A + 1>::run(P, s, i, j, f, g, h);
  }
};

// Populations arriving at node (i, j).  pre: the buffer holds f^ itself
// (right after seeding), so the node reads its own slots.  interior: the
// whole tile is at least one node away from every side, so no rule applies.
template <typename R, int F>
__device__ inline void load_node(const InstP& P, const R* __restrict__ s, int i, int j,
                                 bool interior, bool pre, R* f, R* g, R* h) {
  const int nz = P.nz, pl = P.plane;
  const R* sg = s + 9 * pl;
  const R* sh = s + ((F & F_SWIRL) ? 13 : 9) * pl;
  if (pre) {
    const int o = j * nz + i;
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = s[a * pl + o];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (F & F_SWIRL) g[a] = sg[a * pl + o];
      if (F & F_THERMAL) h[a] = sh[a * pl + o];
    }
  } else if (interior) {
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = s[a * pl + (j - er9(a)) * nz + (i - ez9(a))];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int o = (j - er4(a)) * nz + (i - ez4(a));
      if (F & F_SWIRL) g[a] = sg[a * pl + o];
      if (F & F_THERMAL) h[a] = sh[a * pl + o];
    }
  } else {
    EdgeLoader<R, F, 0>::run(P, s, i, j, f, g, h);
  }
}

}  // namespace lbx
