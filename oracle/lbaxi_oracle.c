/*
 * lbaxi_oracle.c -- plain FP64 CPU oracle of the improved axisymmetric
 * lattice Boltzmann scheme (Li, He, Tang, Tao, "Improved axisymmetric lattice
 * Boltzmann scheme", arXiv:1003.0282).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the GPU path can be
 * checked against something slow and obviously correct.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library: every
 * constant below is written out here from the paper.
 *
 * Conventions (all lattice units, dt = dx = c = 1, cs^2 = 1/3):
 *   node (i, j): i = 0..nz-1 along z (axial), j = 0..nr-1 along r (radial),
 *   r_j = r0 + j.  Array index of population a at node (i, j):
 *   (a*nr + j)*nz + i.  The state held between steps is the pre-collision
 *   population f^ (the paper's f-hat of Eq. 13) plus g (Eq. 53) and h.
 *   tau, tau_g, tau_h are the paper's relaxation parameters (nu = tau/3,
 *   omega0 = 1/(tau + 1/2), Sec. III A); callers holding the usual BGK
 *   relaxation time tau_s convert with tau = tau_s - 1/2.
 *
 * What each function follows:
 *   feq9         Eq. (6)                      D2Q9 equilibrium
 *   geq4         Eq. (54)                     D2Q4 swirl equilibrium, rho -> rho0
 *   heq4         temperature analogue of Eq. (54) (the paper defines no
 *                temperature equation; this reading is an assumption)
 *   node_macros  Eqs. (14)-(17) with mu -> mu0, body force added to F_i
 *   node_source  Eq. (12) (+ centrifugal force rho0 u_th^2 / r, Sec. III C)
 *   node_collide Eq. (13) for f, Eq. (53) for g, its analogue for h
 *   mrt_basis, mrt_source_moments, node_collide_f_mrt
 *                the MRT model of Sec. III B: moments Eq. (38)-(39),
 *                collision Eq. (41) on f-bar = f - S/2 (Eq. 40), source
 *                Eq. (51) plus the mass source, momentum rows modified by
 *                Eqs. (49)-(50); macros are Eqs. (16)-(17) with f-bar
 *   stream       the left-hand side of Eq. (13) / (53): pull streaming, with
 *                periodic ends, specular reflection on the axis (Sec. IV A),
 *                halfway bounce-back / moving walls, free slip
 *   residual     Eq. (57)
 *   *_orig       the original scheme of Sec. II (Eqs. 7-10) that the paper
 *                improves on, with lagged central-difference gradients
 * At r = 0 every term carrying 1/r is taken as zero (Sec. IV A).
 *
 * Parity of the temperature row is unpinned by the paper (it defines no
 * temperature scheme); its pins are closed-form conduction solutions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- lattice (Eq. 6 and the D2Q4 set of Sec. III C) -------------------- */
/* D2Q9 velocities, components (e_z, e_r). */
static const int EZ9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int ER9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* D2Q4 velocities: (1,0), (0,1), (-1,0), (0,-1); weights 1/4. */
static const int EZ4[4] = {1, 0, -1, 0};
static const int ER4[4] = {0, 1, 0, -1};

/* Direction that has e reversed, e_r flipped, e_z flipped: found by search so
 * that no hand-typed permutation table can hide a mistake. */
static int find9(int ez, int er) {
  for (int a = 0; a < 9; ++a)
    if (EZ9[a] == ez && ER9[a] == er) return a;
  return -1;
}
static int find4(int ez, int er) {
  for (int a = 0; a < 4; ++a)
    if (EZ4[a] == ez && ER4[a] == er) return a;
  return -1;
}
static int opp9(int a) { return find9(-EZ9[a], -ER9[a]); }
static int mirr9(int a) { return find9(EZ9[a], -ER9[a]); }
static int mirz9(int a) { return find9(-EZ9[a], ER9[a]); }
static int opp4(int a) { return find4(-EZ4[a], -ER4[a]); }
static int mirr4(int a) { return find4(EZ4[a], -ER4[a]); }

/* ---- parameters -------------------------------------------------------- */
enum { ORC_AXIS = 0, ORC_WALL = 1, ORC_PERIODIC = 2, ORC_FREESLIP = 3 };

typedef struct {
  int kind;           /* ORC_AXIS / ORC_WALL / ORC_PERIODIC / ORC_FREESLIP */
  double uz, ur;      /* wall velocity in the meridian plane */
  double omega;       /* wall angular speed: u_theta at the wall = omega*r */
  int thermal;        /* 0 adiabatic, 1 fixed temperature T */
  double T;
  double r_split;     /* z-walls only: second segment where r_j > r_split */
  int kind2;          /* (r_split < 0 disables the second segment) */
  double omega2;
  int thermal2;
  double T2;
} orc_side;

typedef struct {
  int nz, nr;
  double r0;          /* r_j = r0 + j; r0 = 0 puts the axis on node row 0 */
  int swirl, thermal, cartesian;
  int wet;            /* 1: wall sides are wet-node walls (see wet_substitute) */
  double tau, tau_g, tau_h; /* paper convention */
  double rho0;
  double a0, period, phase; /* axial force density a(t) */
  double gbeta, T_ref;      /* Boussinesq buoyancy rho0*g*beta*(T - T_ref) */
  orc_side side[4];         /* 0 south (r = r0 - 1/2 or axis), 1 north,
                               2 west (z = -1/2), 3 east (z = nz - 1/2) */
  int mrt;                  /* 1: f collides with the MRT model (Sec. III B) */
  double s_e, s_eps, s_q;   /* MRT rates of e, epsilon and q (s_v = 1/(tau+1/2)) */
  double s_rho, s_j;        /* rates of the conserved moments (they drop out) */
  int original;             /* 1: the original scheme of Eqs. (5)-(10), f only */
  int zou_he;               /* 1 (with wet): radial walls rebuild f by Zou-He */
} orc_params;

typedef struct {
  orc_params p;
  double *f, *g, *h;    /* state f^(t), g(t), h(t) */
  double *fs, *gs, *hs; /* post-collision f*, g*, h* (step scratch) */
  double *spd;          /* |u| at the previous time level */
  double *uzp, *urp;    /* original scheme: velocity of the last collided level */
  double *uzn, *urn;    /* (and of the level being collided) */
  int have_spd;
  int64_t t;
} orc_state;

/* ---- small helpers ------------------------------------------------------ */
static double r_of(const orc_params* p, int j) { return p->r0 + (double)j; }
/* 1/r, taken as zero on the axis and in the planar (Cartesian) test mode. */
static double inv_r(const orc_params* p, int j) {
  double r = r_of(p, j);
  if (p->cartesian || r <= 0.0) return 0.0;
  return 1.0 / r;
}
/* Thread the row loops only when the lattice is big enough to pay for it. */
static int par_ok(const orc_params* p) {
  return (long)p->nz * (long)p->nr >= 2048;
}
static int is_axis_row(const orc_params* p, int j) {
  return j == 0 && p->side[0].kind == ORC_AXIS;
}
static size_t IDX(const orc_params* p, int a, int j, int i) {
  return ((size_t)a * (size_t)p->nr + (size_t)j) * (size_t)p->nz + (size_t)i;
}

/* Axial force density at integer time t (periodic when period > 0). */
double orc_force_a(const orc_params* p, int64_t t) {
  if (p->period > 0.0)
    return p->a0 * cos(2.0 * M_PI * (double)t / p->period + p->phase);
  return p->a0;
}

/* ---- equilibria ----------------------------------------------------------- */
/* Eq. (6): f_eq = w rho [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u^2/(2 cs^2)]. */
void orc_feq9(double rho, double uz, double ur, double* out) {
  const double cs2 = 1.0 / 3.0;
  double uu = uz * uz + ur * ur;
  for (int a = 0; a < 9; ++a) {
    double eu = EZ9[a] * uz + ER9[a] * ur;
    out[a] = W9[a] * rho *
             (1.0 + eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

/* Eq. (54): g_eq = (rho u_th / 4)[1 + 2 e.u / c^2]; rho -> rho0 (Sec. III C). */
void orc_geq4(double rho0, double uth, double uz, double ur, double* out) {
  for (int a = 0; a < 4; ++a) {
    double eu = EZ4[a] * uz + ER4[a] * ur;
    out[a] = rho0 * uth / 4.0 * (1.0 + 2.0 * eu);
  }
}

/* Temperature equilibrium built like Eq. (54) with T in place of rho0*u_th. */
void orc_heq4(double T, double uz, double ur, double* out) {
  for (int a = 0; a < 4; ++a) {
    double eu = EZ4[a] * uz + ER4[a] * ur;
    out[a] = T / 4.0 * (1.0 + 2.0 * eu);
  }
}

/* ---- macroscopic variables (Eqs. 14-17) ----------------------------------
 * Eq. (15) with the force split as F_i = G_i - 2 mu0 u_i delta_ir / r^2, where
 * G = (a(t) + rho0 g beta (T - T_ref), rho0 u_th^2 / r) holds every part of
 * the force that does not depend on (u_z, u_r).  Multiplying Eq. (14) by u_i
 * and subtracting it from Eq. (15) gives
 *     u_i (sum f + mu0 delta_ir / r^2) = sum e_i f + G_i / 2,
 * which is Eq. (16) with the body force added; Eq. (17) is unchanged.
 * out = {rho, u_z, u_r, u_th, T}.  g_in must already carry the axis
 * substitution (see node_axis_g) when j is the axis row.                    */
void orc_node_macros(const orc_params* p, int j, int64_t t, const double* fh,
                     const double* g, const double* h, double* out) {
  double ir = inv_r(p, j);
  double mu0 = p->rho0 * p->tau / 3.0; /* mu = tau rho cs^2 dt, Eq. (36) */
  double s0 = 0, sz = 0, sr = 0;
  for (int a = 0; a < 9; ++a) {
    s0 += fh[a];
    sz += EZ9[a] * fh[a];
    sr += ER9[a] * fh[a];
  }
  double uth = 0.0, T = p->T_ref;
  if (p->swirl) {
    double sg = 0;
    for (int a = 0; a < 4; ++a) sg += g[a];
    uth = is_axis_row(p, j) ? 0.0 : sg / p->rho0; /* u_th = sum g / rho0 */
  }
  if (p->thermal) {
    T = 0;
    for (int a = 0; a < 4; ++a) T += h[a];
  }
  double Gz = orc_force_a(p, t);
  if (p->thermal) Gz += p->rho0 * p->gbeta * (T - p->T_ref);
  double Gr = p->swirl ? p->rho0 * uth * uth * ir : 0.0;
  double ur = (sr + 0.5 * Gr) / (s0 + mu0 * ir * ir); /* Eq. (16), i = r */
  double rho = s0 / (1.0 + 0.5 * ur * ir);           /* Eq. (17) */
  double uz = (sz + 0.5 * Gz) / s0;                   /* Eq. (16), i = z */
  out[0] = rho;
  out[1] = uz;
  out[2] = ur;
  out[3] = uth;
  out[4] = T;
}

/* Force of Eq. (12) at a node with macros m: F_z = a(t) (+ buoyancy) and
 * F_r = -2 mu0 u_r / r^2 + rho0 u_th^2 / r. */
static void node_force(const orc_params* p, int j, int64_t t, const double* m,
                       double* Fz, double* Fr) {
  double ir = inv_r(p, j);
  double mu0 = p->rho0 * p->tau / 3.0;
  double uz = m[1], ur = m[2], uth = m[3], T = m[4];
  (void)uz;
  *Fz = orc_force_a(p, t);
  if (p->thermal) *Fz += p->rho0 * p->gbeta * (T - p->T_ref);
  *Fr = -2.0 * mu0 * ur * ir * ir;
  if (p->swirl) *Fr += p->rho0 * uth * uth * ir;
}

static void node_source_mrt(const orc_params* p, int j, int64_t t,
                            const double* m, const double* feq, double* S);

/* Eq. (12): S_a = [(e_ai - u_i) F_i / (rho cs^2) - u_r / r] f_eq_a with
 * F_r = -2 mu0 u_r / r^2 + rho0 u_th^2 / r and F_z = a(t) (+ buoyancy).
 * With the MRT model the source is the one of Sec. III B instead. */
void orc_node_source(const orc_params* p, int j, int64_t t, const double* m,
                     const double* feq, double* S) {
  if (p->mrt) {
    node_source_mrt(p, j, t, m, feq, S);
    return;
  }
  double ir = inv_r(p, j);
  const double cs2 = 1.0 / 3.0;
  double rho = m[0], uz = m[1], ur = m[2];
  double Fz, Fr;
  node_force(p, j, t, m, &Fz, &Fr);
  for (int a = 0; a < 9; ++a) {
    double eF = (EZ9[a] - uz) * Fz + (ER9[a] - ur) * Fr;
    S[a] = (eF / (rho * cs2) - ur * ir) * feq[a];
  }
}

/* Axis treatment of g (non-equilibrium extrapolation, Sec. IV B): the swirl
 * population on the axis node becomes the non-equilibrium part of its radial
 * neighbour, g(i,0) = g(i,1) - g_eq(i,1), with row-1 macros at the same time
 * level; u_th vanishes on the axis. */
static void node_axis_g(const orc_params* p, int64_t t, const double* f1,
                        const double* g1, const double* h1, double* g0) {
  double m1[5], geq1[4];
  orc_node_macros(p, 1, t, f1, g1, h1, m1);
  orc_geq4(p->rho0, m1[3], m1[1], m1[2], geq1);
  for (int a = 0; a < 4; ++a) g0[a] = g1[a] - geq1[a];
}

/* ---- MRT collision (Sec. III B) ----------------------------------------------
 * The moments of Eq. (38) with x = r and y = z (the paper pairs (r, z) with
 * (x, y)).  Row k of M is a polynomial in the velocity components evaluated on
 * the nine D2Q9 velocities:
 *   rho  1                      e    -4 + 3|e|^2
 *   eps  4 - 21|e|^2/2 + 9|e|^4/2
 *   j_x  e_x                    q_x  (-5 + 3|e|^2) e_x
 *   j_y  e_y                    q_y  (-5 + 3|e|^2) e_y
 *   p_xx e_x^2 - e_y^2          p_xy e_x e_y
 * The rows are mutually orthogonal (the basis of the paper's Ref. 9), so
 * M^-1 = M^T diag(1 / |row k|^2).  M is row-major [k][a], M^-1 [a][k].     */
void orc_mrt_basis(double* M, double* Minv) {
  for (int a = 0; a < 9; ++a) {
    double ex = ER9[a], ey = EZ9[a], e2 = ex * ex + ey * ey;
    double row[9] = {1.0,
                     -4.0 + 3.0 * e2,
                     4.0 - 10.5 * e2 + 4.5 * e2 * e2,
                     ex,
                     (-5.0 + 3.0 * e2) * ex,
                     ey,
                     (-5.0 + 3.0 * e2) * ey,
                     ex * ex - ey * ey,
                     ex * ey};
    for (int k = 0; k < 9; ++k) M[k * 9 + a] = row[k];
  }
  for (int k = 0; k < 9; ++k) {
    double n2 = 0.0;
    for (int a = 0; a < 9; ++a) n2 += M[k * 9 + a] * M[k * 9 + a];
    for (int a = 0; a < 9; ++a) Minv[a * 9 + k] = M[k * 9 + a] / n2;
  }
}

static void matvec9(const double* A, const double* x, double* y) {
  for (int r = 0; r < 9; ++r) {
    double s = 0.0;
    for (int c = 0; c < 9; ++c) s += A[r * 9 + c] * x[c];
    y[r] = s;
  }
}

/* Source in moment space: S~ = -(u_r / r) m_eq + S~' with S~' of Eq. (51),
 * F_x = F_r and F_y = F_z of Eq. (12).  The mass part carries the sign of
 * Eq. (12)'s -(u_r / r) f_eq, so that the zeroth moment of the source is the
 * continuity source -rho u_r / r of Eq. (1).  m holds the macros {rho, u_z,
 * u_r, u_th, T} and meq = M f_eq. */
void orc_mrt_source_moments(const orc_params* p, int j, int64_t t,
                            const double* m, const double* meq, double* St) {
  double ir = inv_r(p, j);
  double Fz, Fr;
  node_force(p, j, t, m, &Fz, &Fr);
  double ux = m[2], uy = m[1], Fx = Fr, Fy = Fz;
  double uF = ux * Fx + uy * Fy;
  double Sp[9] = {0.0,  6.0 * uF, -6.0 * uF, Fx, -Fx, Fy, -Fy,
                  2.0 * (ux * Fx - uy * Fy), ux * Fy + uy * Fx};
  for (int k = 0; k < 9; ++k) St[k] = -m[2] * ir * meq[k] + Sp[k];
}

/* The source in velocity space, S = M^-1 S~: the equilibrium of the f-bar
 * variables is f_eq - S/2 (f-bar = f - S/2, Eq. 40). */
static void node_source_mrt(const orc_params* p, int j, int64_t t,
                            const double* m, const double* feq, double* S) {
  double M[81], Minv[81], meq[9], St[9];
  orc_mrt_basis(M, Minv);
  matvec9(M, feq, meq);
  orc_mrt_source_moments(p, j, t, m, meq, St);
  matvec9(Minv, St, S);
}

/* Collision of f-bar in moment space, Eq. (41), with the momentum rows
 * modified by Eqs. (49)-(50); the result f-bar+ = M^-1 m-bar+ is what Eq.
 * (42) streams.  Lambda = diag(s_rho, s_e, s_eps, s_j, s_q, s_j, s_q, s_v,
 * s_v) with s_v = 1 / (tau + 1/2) (mu = (1/s_v - 1/2) rho / 3).  In Eqs.
 * (49)-(50) m^(1) = (m-bar - m_eq) + S~/2 and gamma = (1 - s_v/2) / r, which
 * is zero wherever 1/r is taken as zero.                                    */
static void node_collide_f_mrt(const orc_params* p, int j, int64_t t,
                               const double* fb, const double* m, double* fo) {
  double M[81], Minv[81], feq[9], meq[9], mb[9], St[9], mp[9];
  orc_mrt_basis(M, Minv);
  orc_feq9(m[0], m[1], m[2], feq);
  matvec9(M, feq, meq);
  matvec9(M, fb, mb);
  orc_mrt_source_moments(p, j, t, m, meq, St);
  double sv = 1.0 / (p->tau + 0.5);
  double s[9] = {p->s_rho, p->s_e, p->s_eps, p->s_j, p->s_q,
                 p->s_j,   p->s_q, sv,       sv};
  for (int k = 0; k < 9; ++k)
    mp[k] = mb[k] - s[k] * (mb[k] - meq[k]) + (1.0 - 0.5 * s[k]) * St[k];
  double e1 = mb[1] - meq[1] + 0.5 * St[1];
  double pxx1 = mb[7] - meq[7] + 0.5 * St[7];
  double pxy1 = mb[8] - meq[8] + 0.5 * St[8];
  double gam = (1.0 - 0.5 * sv) * inv_r(p, j);
  mp[3] -= gam * (p->s_e / (6.0 * sv) * e1 + 0.5 * pxx1); /* Eq. (49) */
  mp[5] -= gam * pxy1;                                     /* Eq. (50) */
  matvec9(Minv, mp, fo);
}

/* Eq. (13) for f (or the MRT collision above), Eq. (53) for g and the
 * analogous rule for h, at one node.  Inputs are the pre-collision
 * populations (g already axis-substituted); outputs are the post-collision
 * populations and the macros m[5].                                          */
void orc_node_collide(const orc_params* p, int j, int64_t t, const double* fh,
                      const double* g, const double* h, double* fo, double* go,
                      double* ho, double* m) {
  double ir = inv_r(p, j);
  orc_node_macros(p, j, t, fh, g, h, m);
  double rho = m[0], uz = m[1], ur = m[2], uth = m[3], T = m[4];
  if (p->mrt) {
    node_collide_f_mrt(p, j, t, fh, m, fo);
  } else {
    double feq[9], S[9];
    orc_feq9(rho, uz, ur, feq);
    orc_node_source(p, j, t, m, feq, S);
    for (int a = 0; a < 9; ++a) {
      /* omega_f = [1 + tau e_ar / r] / (tau + 0.5), after Eq. (13) */
      double w = (1.0 + p->tau * ER9[a] * ir) / (p->tau + 0.5);
      fo[a] = fh[a] - w * (fh[a] - feq[a]) + (1.0 - 0.5 * w) * S[a];
    }
  }
  if (p->swirl) {
    double geq[4];
    orc_geq4(p->rho0, uth, uz, ur, geq);
    double nu = p->tau_g / 2.0; /* nu = tau_g c^2 / 2 */
    for (int a = 0; a < 4; ++a) {
      double w = (1.0 + p->tau_g * ER4[a] * ir) / (p->tau_g + 0.5);
      double Sg = -ir * (2.0 * ur + nu * ir) * geq[a]; /* Eq. (54) */
      go[a] = g[a] - w * (g[a] - geq[a]) + Sg;
    }
  }
  if (p->thermal) {
    double heq[4];
    orc_heq4(T, uz, ur, heq);
    for (int a = 0; a < 4; ++a) {
      double w = (1.0 + p->tau_h * ER4[a] * ir) / (p->tau_h + 0.5);
      double Sh = -ur * ir * heq[a];
      ho[a] = h[a] - w * (h[a] - heq[a]) + Sh;
    }
  }
}

/* ---- the original scheme (Sec. II, Eqs. 5-10) ---------------------------------
 * Premnath and Abraham's scheme as the paper restates it: f~ = f - Omega/2 -
 * G/2 collides by Eq. (8) with the constant rate omega = 1/(tau + 1/2) and
 * the source of Eq. (7),
 *   G_a = -w_a rho u_r / r + (e_a - u).F / (rho cs^2) f_eq_a,
 *   F_i = (mu / r) D_i - 2 mu u_i delta_ir / r^2 - rho u_i u_r / r
 *         (+ the body force along z),
 * with D_r = 2 d_r u_r and D_z = d_r u_z + d_z u_r; the macros are Eqs.
 * (9)-(10).  mu -> mu0 as in the improved scheme.  The paper gives no
 * stencil for D: D is supplied by the caller (see lagged_grad).  With D
 * known, Eqs. (9)-(10) solve explicitly: s0 = sum f~ = rho (1 + u_r / 2r),
 *   u_r = (sum e_r f~ + mu0 D_r / 2r) / (s0 + mu0 / r^2),
 *   u_z = (sum e_z f~ + mu0 D_z / 2r + a / 2) / s0,  rho = s0 / (1 + u_r / 2r).
 * Only f is modelled (no swirl or temperature fields in this scheme).       */
void orc_node_macros_orig(const orc_params* p, int j, int64_t t,
                          const double* fh, double Dr, double Dz, double* out) {
  double ir = inv_r(p, j);
  double mu0 = p->rho0 * p->tau / 3.0;
  double s0 = 0, sz = 0, sr = 0;
  for (int a = 0; a < 9; ++a) {
    s0 += fh[a];
    sz += EZ9[a] * fh[a];
    sr += ER9[a] * fh[a];
  }
  double ur = (sr + 0.5 * mu0 * Dr * ir) / (s0 + mu0 * ir * ir);
  double uz = (sz + 0.5 * (mu0 * Dz * ir + orc_force_a(p, t))) / s0;
  out[0] = s0 / (1.0 + 0.5 * ur * ir);
  out[1] = uz;
  out[2] = ur;
  out[3] = 0.0;
  out[4] = p->T_ref;
}

/* Eq. (7) at a node with macros m and gradient terms D. */
void orc_node_source_orig(const orc_params* p, int j, int64_t t,
                          const double* m, double Dr, double Dz,
                          const double* feq, double* G) {
  double ir = inv_r(p, j);
  double mu0 = p->rho0 * p->tau / 3.0;
  const double cs2 = 1.0 / 3.0;
  double rho = m[0], uz = m[1], ur = m[2];
  double Fr = mu0 * ir * Dr - 2.0 * mu0 * ur * ir * ir - rho * ur * ur * ir;
  double Fz = mu0 * ir * Dz - rho * uz * ur * ir + orc_force_a(p, t);
  for (int a = 0; a < 9; ++a) {
    double eF = (EZ9[a] - uz) * Fz + (ER9[a] - ur) * Fr;
    G[a] = -W9[a] * rho * ur * ir + eF / (rho * cs2) * feq[a];
  }
}

/* Eq. (8) at one node: macros (Eqs. 9-10), then the BGK update with the
 * constant rate and the source of Eq. (7). */
void orc_node_collide_orig(const orc_params* p, int j, int64_t t,
                           const double* fh, double Dr, double Dz, double* fo,
                           double* m) {
  double feq[9], G[9];
  orc_node_macros_orig(p, j, t, fh, Dr, Dz, m);
  orc_feq9(m[0], m[1], m[2], feq);
  orc_node_source_orig(p, j, t, m, Dr, Dz, feq, G);
  double w = 1.0 / (p->tau + 0.5);
  for (int a = 0; a < 9; ++a)
    fo[a] = fh[a] - w * (fh[a] - feq[a]) + (1.0 - 0.5 * w) * G[a];
}

/* ---- boundaries ------------------------------------------------------------
 * A wall lies half a lattice spacing outside the last fluid node.  A
 * population whose upstream node lies outside the domain takes the rule of the
 * boundary it crossed; a z-end is checked before the radial sides. */
typedef struct { int kind; double omega; int thermal; double T; } seg_t;

typedef struct {
  int in, jn;      /* inner neighbour */
  int free;        /* free-slip segment */
  double uz, ur;   /* wall velocity in the meridian plane */
  double omega;    /* wall angular speed */
  int thermal;
  double T;
} wet_rule_t;

static seg_t zwall_segment(const orc_params* p, const orc_side* s, int j) {
  seg_t sg;
  if (s->r_split >= 0.0 && r_of(p, j) > s->r_split) {
    sg.kind = s->kind2; sg.omega = s->omega2; sg.thermal = s->thermal2;
    sg.T = s->T2;
  } else {
    sg.kind = s->kind; sg.omega = s->omega; sg.thermal = s->thermal;
    sg.T = s->T;
  }
  return sg;
}

/* Moving-wall bounce-back term 6 w_a rho0 (e_a . u_w). */
static double wall_term9(const orc_params* p, const orc_side* s, int a) {
  return 6.0 * W9[a] * p->rho0 * (EZ9[a] * s->uz + ER9[a] * s->ur);
}

static double pull_f(const orc_params* p, const double* fs, int i, int j,
                     int a) {
  int iz = i - EZ9[a], jr = j - ER9[a];
  if (iz < 0 || iz >= p->nz) {
    const orc_side* s = &p->side[iz < 0 ? 2 : 3];
    if (s->kind == ORC_PERIODIC) {
      iz = (iz + p->nz) % p->nz;
    } else {
      seg_t sg = zwall_segment(p, s, j);
      if (sg.kind == ORC_FREESLIP) {
        /* specular reflection on the z-end: arrives from (i, j - e_r) with
         * e_z reversed */
        int j2 = j - ER9[a], b = mirz9(a);
        if (j2 >= 0 && j2 < p->nr) return fs[IDX(p, b, j2, i)];
        if (j2 < 0 && p->side[0].kind == ORC_AXIS)
          return fs[IDX(p, mirr9(b), 1, i)];
        return fs[IDX(p, opp9(a), j, i)];
      }
      return fs[IDX(p, opp9(a), j, i)] + wall_term9(p, s, a);
    }
  }
  if (jr < 0) {
    const orc_side* s = &p->side[0];
    if (s->kind == ORC_AXIS) /* ghost (iz,-1) is the mirror image of (iz,1) */
      return fs[IDX(p, mirr9(a), 1, iz)];
    return fs[IDX(p, opp9(a), j, i)] + wall_term9(p, s, a);
  }
  if (jr >= p->nr) {
    const orc_side* s = &p->side[1];
    return fs[IDX(p, opp9(a), j, i)] + wall_term9(p, s, a);
  }
  return fs[IDX(p, a, jr, iz)];
}

static double pull_g(const orc_params* p, const double* gs, int i, int j,
                     int a) {
  int iz = i - EZ4[a], jr = j - ER4[a];
  if (iz < 0 || iz >= p->nz) {
    const orc_side* s = &p->side[iz < 0 ? 2 : 3];
    if (s->kind == ORC_PERIODIC) {
      iz = (iz + p->nz) % p->nz;
    } else {
      seg_t sg = zwall_segment(p, s, j);
      if (sg.kind == ORC_FREESLIP) return gs[IDX(p, opp4(a), j, i)];
      /* anti-bounce-back, rho0 u_th = rho0 omega r at the wall */
      return -gs[IDX(p, opp4(a), j, i)] + 0.5 * p->rho0 * sg.omega * r_of(p, j);
    }
  }
  if (jr < 0) {
    const orc_side* s = &p->side[0];
    if (s->kind == ORC_AXIS) return 0.0; /* replaced on the axis, see above */
    double rw = p->r0 - 0.5;
    return -gs[IDX(p, opp4(a), j, i)] + 0.5 * p->rho0 * s->omega * rw;
  }
  if (jr >= p->nr) {
    const orc_side* s = &p->side[1];
    double rw = p->r0 + (double)p->nr - 0.5;
    return -gs[IDX(p, opp4(a), j, i)] + 0.5 * p->rho0 * s->omega * rw;
  }
  return gs[IDX(p, a, jr, iz)];
}

static double pull_h(const orc_params* p, const double* hs, int i, int j,
                     int a) {
  int iz = i - EZ4[a], jr = j - ER4[a];
  if (iz < 0 || iz >= p->nz) {
    const orc_side* s = &p->side[iz < 0 ? 2 : 3];
    if (s->kind == ORC_PERIODIC) {
      iz = (iz + p->nz) % p->nz;
    } else {
      seg_t sg = zwall_segment(p, s, j);
      if (sg.kind == ORC_WALL && sg.thermal)
        return -hs[IDX(p, opp4(a), j, i)] + 0.5 * sg.T;
      return hs[IDX(p, opp4(a), j, i)]; /* adiabatic */
    }
  }
  if (jr < 0) {
    const orc_side* s = &p->side[0];
    if (s->kind == ORC_AXIS) return hs[IDX(p, mirr4(a), 1, iz)];
    if (s->thermal) return -hs[IDX(p, opp4(a), j, i)] + 0.5 * s->T;
    return hs[IDX(p, opp4(a), j, i)];
  }
  if (jr >= p->nr) {
    const orc_side* s = &p->side[1];
    if (s->thermal) return -hs[IDX(p, opp4(a), j, i)] + 0.5 * s->T;
    return hs[IDX(p, opp4(a), j, i)];
  }
  return hs[IDX(p, a, jr, iz)];
}

/* ---- state management ------------------------------------------------------ */
static size_t nodes(const orc_params* p) {
  return (size_t)p->nz * (size_t)p->nr;
}

orc_state* orc_create(const orc_params* p) {
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  if (!s) return NULL;
  s->p = *p;
  size_t n = nodes(p);
  s->f = (double*)calloc(9 * n, sizeof(double));
  s->fs = (double*)calloc(9 * n, sizeof(double));
  s->g = (double*)calloc(4 * n, sizeof(double));
  s->gs = (double*)calloc(4 * n, sizeof(double));
  s->h = (double*)calloc(4 * n, sizeof(double));
  s->hs = (double*)calloc(4 * n, sizeof(double));
  s->spd = (double*)calloc(n, sizeof(double));
  s->uzp = (double*)calloc(n, sizeof(double));
  s->urp = (double*)calloc(n, sizeof(double));
  s->uzn = (double*)calloc(n, sizeof(double));
  s->urn = (double*)calloc(n, sizeof(double));
  if (!s->f || !s->fs || !s->g || !s->gs || !s->h || !s->hs || !s->spd ||
      !s->uzp || !s->urp || !s->uzn || !s->urn) {
    free(s->f); free(s->fs); free(s->g); free(s->gs); free(s->h);
    free(s->hs); free(s->spd); free(s->uzp); free(s->urp); free(s->uzn);
    free(s->urn); free(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_state* s) {
  if (!s) return;
  free(s->f); free(s->fs); free(s->g); free(s->gs); free(s->h);
  free(s->hs); free(s->spd); free(s->uzp); free(s->urp); free(s->uzn);
  free(s->urn); free(s);
}

int64_t orc_time(const orc_state* s) { return s->t; }

/* Gather the populations of node (i, j) from the state arrays. */
static void gather(const orc_state* s, int i, int j, double* f, double* g,
                   double* h) {
  const orc_params* p = &s->p;
  for (int a = 0; a < 9; ++a) f[a] = s->f[IDX(p, a, j, i)];
  for (int a = 0; a < 4; ++a) {
    g[a] = p->swirl ? s->g[IDX(p, a, j, i)] : 0.0;
    h[a] = p->thermal ? s->h[IDX(p, a, j, i)] : 0.0;
  }
}

/* Populations at (i, j) ready for the macros: on the axis row the swirl
 * populations are replaced by the extrapolated ones. */
static int wet_wall_rule(const orc_params* p, int i, int j, wet_rule_t* w);

static void node_inputs(const orc_state* s, int i, int j, double* f, double* g,
                        double* h) {
  gather(s, i, j, f, g, h);
  if (s->p.swirl && is_axis_row(&s->p, j) && !wet_wall_rule(&s->p, i, j, NULL)) {
    double f1[9], g1[4], h1[4];
    gather(s, i, 1, f1, g1, h1);
    node_axis_g(&s->p, s->t, f1, g1, h1, g);
  }
}

/* Velocity of node (i, j) of the field (uz, ur), for i in [-1, nz] and j in
 * [-1, nr] (never both outside): ghost values are mirrored across the axis
 * (u_r odd) and across a free-slip end (u_z odd), wrapped at periodic ends,
 * and 2 u_w - u beyond a halfway wall (linear through the wall, which lies
 * half a spacing out). */
static void vel_at(const orc_params* p, const double* uz, const double* ur,
                   int i, int j, double* vz, double* vr) {
  if (i < 0 || i >= p->nz) {
    const orc_side* s = &p->side[i < 0 ? 2 : 3];
    int in = i < 0 ? 0 : p->nz - 1;
    if (s->kind == ORC_PERIODIC) {
      int iw = (i + p->nz) % p->nz;
      *vz = uz[(size_t)j * p->nz + iw];
      *vr = ur[(size_t)j * p->nz + iw];
      return;
    }
    double z0 = uz[(size_t)j * p->nz + in], r0v = ur[(size_t)j * p->nz + in];
    seg_t sg = zwall_segment(p, s, j);
    if (sg.kind == ORC_FREESLIP) {
      *vz = -z0;
      *vr = r0v;
    } else {
      *vz = 2.0 * s->uz - z0;
      *vr = 2.0 * s->ur - r0v;
    }
    return;
  }
  if (j < 0) {
    const orc_side* s = &p->side[0];
    if (s->kind == ORC_AXIS) {
      *vz = uz[(size_t)1 * p->nz + i];
      *vr = -ur[(size_t)1 * p->nz + i];
    } else {
      *vz = 2.0 * s->uz - uz[i];
      *vr = 2.0 * s->ur - ur[i];
    }
    return;
  }
  if (j >= p->nr) {
    const orc_side* s = &p->side[1];
    size_t o = (size_t)(p->nr - 1) * p->nz + i;
    *vz = 2.0 * s->uz - uz[o];
    *vr = 2.0 * s->ur - ur[o];
    return;
  }
  *vz = uz[(size_t)j * p->nz + i];
  *vr = ur[(size_t)j * p->nz + i];
}

/* The gradient terms of Eq. (7), D_r = 2 d_r u_r and D_z = d_r u_z + d_z u_r,
 * by second-order central differences of the given velocity field (the
 * paper gives no stencil).  They enter only multiplied by 1/r, so they are
 * zero where 1/r is taken as zero. */
static void grad_terms(const orc_params* p, const double* uz, const double* ur,
                       int i, int j, double* Dr, double* Dz) {
  *Dr = 0.0;
  *Dz = 0.0;
  if (inv_r(p, j) == 0.0) return;
  double zn, rn, zs, rs, ze, re, zw, rw;
  vel_at(p, uz, ur, i, j + 1, &zn, &rn);
  vel_at(p, uz, ur, i, j - 1, &zs, &rs);
  vel_at(p, uz, ur, i + 1, j, &ze, &re);
  vel_at(p, uz, ur, i - 1, j, &zw, &rw);
  *Dr = rn - rs;                          /* 2 (rn - rs) / 2 */
  *Dz = 0.5 * (zn - zs) + 0.5 * (re - rw);
}

/* Equilibrium seeding: f^ = f_eq(rho, u) - S(rho, u)/2 (the paper's
 * f^ = f - Omega/2 - S/2 with Omega = 0), g = g_eq, h = h_eq.  NULL fields
 * mean rho0 / zero velocity / T_ref.  On the axis row u_r and u_th are forced
 * to 0.  Summing Eq. (12) gives sum S = -rho u_r / r and sum e_r S = F_r -
 * rho u_r^2 / r, so Eqs. (16)-(17) return the seeded rho and u exactly.      */
void orc_seed(orc_state* s, const double* uz, const double* ur,
              const double* uth, const double* T, const double* rho) {
  const orc_params* p = &s->p;
  s->t = 0;
  s->have_spd = 0;
  /* original scheme: the seeded velocity is the field its gradients start from */
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      size_t n = (size_t)j * p->nz + i;
      s->uzp[n] = uz ? uz[n] : 0.0;
      s->urp[n] = (ur && !is_axis_row(p, j)) ? ur[n] : 0.0;
    }
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      size_t n = (size_t)j * p->nz + i;
      double m[5];
      m[0] = rho ? rho[n] : p->rho0;
      m[1] = uz ? uz[n] : 0.0;
      m[2] = ur ? ur[n] : 0.0;
      m[3] = (uth && p->swirl) ? uth[n] : 0.0;
      m[4] = (T && p->thermal) ? T[n] : p->T_ref;
      if (is_axis_row(p, j)) { m[2] = 0.0; m[3] = 0.0; }
      double feq[9], S[9], geq[4], heq[4];
      orc_feq9(m[0], m[1], m[2], feq);
      if (p->original) {
        /* f~ = f_eq - G/2 with D from the seeded velocity field */
        double Dr, Dz;
        grad_terms(p, s->uzp, s->urp, i, j, &Dr, &Dz);
        orc_node_source_orig(p, j, 0, m, Dr, Dz, feq, S);
      } else {
        orc_node_source(p, j, 0, m, feq, S);
      }
      for (int a = 0; a < 9; ++a) s->f[IDX(p, a, j, i)] = feq[a] - 0.5 * S[a];
      if (p->swirl) {
        orc_geq4(p->rho0, m[3], m[1], m[2], geq);
        for (int a = 0; a < 4; ++a) s->g[IDX(p, a, j, i)] = geq[a];
      }
      if (p->thermal) {
        orc_heq4(m[4], m[1], m[2], heq);
        for (int a = 0; a < 4; ++a) s->h[IDX(p, a, j, i)] = heq[a];
      }
    }
}

/* Macroscopic fields of the current state; any output may be NULL. */
/* Macros of node (i, j) at the current level (Eqs. 16-17, or Eqs. 9-10 of
 * the original scheme with D from the last collided level's velocity). */
static void state_macros(const orc_state* s, int i, int j, double* m) {
  double f[9], g[4], h[4];
  node_inputs(s, i, j, f, g, h);
  if (s->p.original) {
    double Dr, Dz;
    grad_terms(&s->p, s->uzp, s->urp, i, j, &Dr, &Dz);
    orc_node_macros_orig(&s->p, j, s->t, f, Dr, Dz, m);
  } else {
    orc_node_macros(&s->p, j, s->t, f, g, h, m);
  }
}

void orc_macros(const orc_state* s, double* rho, double* uz, double* ur,
                double* uth, double* T) {
  const orc_params* p = &s->p;
#pragma omp parallel for schedule(static) if (par_ok(p))
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      double m[5];
      size_t n = (size_t)j * p->nz + i;
      state_macros(s, i, j, m);
      if (rho) rho[n] = m[0];
      if (uz) uz[n] = m[1];
      if (ur) ur[n] = m[2];
      if (uth) uth[n] = m[3];
      if (T) T[n] = m[4];
    }
}

/* Streaming of the post-collision arrays into the state arrays. */
static void stream_all(orc_state* s) {
  const orc_params* p = &s->p;
#pragma omp parallel for schedule(static) if (par_ok(p))
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      for (int a = 0; a < 9; ++a) s->f[IDX(p, a, j, i)] = pull_f(p, s->fs, i, j, a);
      if (p->swirl)
        for (int a = 0; a < 4; ++a) s->g[IDX(p, a, j, i)] = pull_g(p, s->gs, i, j, a);
      if (p->thermal)
        for (int a = 0; a < 4; ++a) s->h[IDX(p, a, j, i)] = pull_h(p, s->hs, i, j, a);
    }
}

/* n time steps t -> t + n: collide every node (Eqs. 12-17, 53-54), then
 * stream.  The speed |u| of each collided level is kept for Eq. (57). */
/* ---- wet-node walls ----------------------------------------------------------
 * The paper treats the walls of its rotating flows by non-equilibrium
 * extrapolation (Sec. IV B, its Ref. 59): the wall passes through the
 * outermost node row or column, and after every streaming step the state of
 * such a wall node b is rebuilt from its inner neighbour n,
 *     f^(b) = E(rho_n, u_w; b) + [f^(n) - E(rho_n, u_n; n)],
 * with E = f_eq - S/2 the equilibrium of the f^ variables (Eqs. 6, 12; the
 * source taken with the wall values at b), and likewise g with the wall
 * value rho0 Omega r_b of rho0 u_th and h with the wall temperature (or T_n
 * on an adiabatic wall), rho_n and u_n being the Eq. (16)-(17) macros of n.
 * Eqs. (16)-(17) then return exactly (rho_n, u_w) at b.  n is one node inward along the wall normal; a
 * node on a z-end and a radial wall takes the z-end's values and its diagonal
 * inner neighbour.  A free-slip z-end segment is a wet node too, with wall
 * velocity (0, u_r,n), u_th,n and T_n (zero normal velocity, no shear, no
 * flux).  Wall nodes keep their own g on the axis row.                     */
static int wet_wall_rule(const orc_params* p, int i, int j, wet_rule_t* w) {
  if (!p->wet) return 0;
  const orc_side* zs = NULL;
  int dz = 0;
  if (i == 0 && p->side[2].kind != ORC_PERIODIC) {
    zs = &p->side[2];
    dz = 1;
  } else if (i == p->nz - 1 && p->side[3].kind != ORC_PERIODIC) {
    zs = &p->side[3];
    dz = -1;
  }
  int north = j == p->nr - 1 && p->side[1].kind == ORC_WALL;
  int south = j == 0 && p->side[0].kind == ORC_WALL;
  if (!zs && !north && !south) return 0;
  if (!w) return 1;
  w->in = i + dz;
  w->jn = j + (north ? -1 : (south ? 1 : 0));
  if (zs) {
    seg_t sg = zwall_segment(p, zs, j);
    w->free = sg.kind == ORC_FREESLIP;
    w->uz = zs->uz; w->ur = zs->ur;
    w->omega = sg.omega; w->thermal = sg.thermal; w->T = sg.T;
  } else {
    const orc_side* rs = &p->side[north ? 1 : 0];
    w->free = 0;
    w->uz = rs->uz; w->ur = rs->ur;
    w->omega = rs->omega; w->thermal = rs->thermal; w->T = rs->T;
  }
  return 1;
}

/* Zou-He no-slip wall (the paper's Ref. 47, used for its pipe flows) for the
 * f^ variables at a node b on a radial wall (north: row nr - 1, south: row
 * 0 of an annulus) whose wall velocity u_w = (u_z,w, 0) has no normal part.
 * The populations that streamed in from the fluid side are kept; the three
 * that would have come from beyond the wall (e_r pointing away from the
 * wall, into the fluid) are fixed by Eqs. (16)-(17) at b with u = u_w,
 *   sum e_r f^ = -G_r / 2,   sum e_z f^ = u_z,w sum f^ - G_z / 2,
 * (G the velocity-independent force of the macros) and by bounce-back of
 * the non-equilibrium part along the wall normal, f^_n - E_n = f^_m - E_m
 * (m the direction opposite to n, E = f_eq - S/2 at the wall state).  The
 * two diagonal unknowns share the remaining mass equally, as in Zou and He.
 * mb holds the wall values (u_z,w, u_r,w = 0, u_th,w, T_w) of b.          */
static void zou_he_f(orc_state* s, int i, int j, const double* mb) {
  const orc_params* p = &s->p;
  int north = (j == p->nr - 1);
  int sgn = north ? -1 : 1;        /* e_r of the unknown directions */
  double f[9];
  for (int a = 0; a < 9; ++a) f[a] = s->f[IDX(p, a, j, i)];
  double Gz = orc_force_a(p, s->t);
  if (p->thermal) Gz += p->rho0 * p->gbeta * (mb[4] - p->T_ref);
  double Gr = p->swirl ? p->rho0 * mb[3] * mb[3] * inv_r(p, j) : 0.0;
  /* known sums: e_r = 0 and e_r = -sgn (arriving from the fluid side) */
  double A0 = 0.0, Ak = 0.0, Zk = 0.0;
  for (int a = 0; a < 9; ++a) {
    if (ER9[a] == 0) {
      A0 += f[a];
      Zk += EZ9[a] * f[a];
    } else if (ER9[a] == -sgn) {
      Ak += f[a];
      Zk += EZ9[a] * f[a];
    }
  }
  /* radial momentum: sgn * U - sgn * Ak = -Gr/2, U the unknowns' sum */
  double U = Ak - sgn * 0.5 * Gr;
  double s0 = A0 + Ak + U;
  /* axial momentum: Zk + sum over unknowns of e_z f = u_z,w s0 - Gz/2 */
  double Dz = mb[1] * s0 - 0.5 * Gz - Zk;
  int n = find9(0, sgn), m = find9(0, -sgn);
  int dp = find9(1, sgn), dm = find9(-1, sgn);  /* e_z = +1 / -1 unknowns */
  /* the wall state takes the density these conditions give, rho = s0
   * (Eq. 17 with u_r = 0) */
  double mz[5] = {s0, mb[1], mb[2], mb[3], mb[4]}, ez[9], Sz[9];
  orc_feq9(mz[0], mz[1], mz[2], ez);
  orc_node_source(p, j, s->t, mz, ez, Sz);
  double fn = f[m] + (ez[n] - 0.5 * Sz[n]) - (ez[m] - 0.5 * Sz[m]);
  s->f[IDX(p, n, j, i)] = fn;
  s->f[IDX(p, dp, j, i)] = 0.5 * (U - fn + Dz);
  s->f[IDX(p, dm, j, i)] = 0.5 * (U - fn - Dz);
}

static void wet_substitute(orc_state* s) {
  const orc_params* p = &s->p;
  if (!p->wet) return;
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      wet_rule_t w;
      if (!wet_wall_rule(p, i, j, &w)) continue;
      double f[9], g[4], h[4], m[5], mb[5], e1[9], e2[9], S1[9], S2[9];
      /* mass of b as streamed in (its links out of the domain bounce back),
       * kept by the substitution so that no mass crosses the wall */
      double s0b = 0.0;
      for (int a = 0; a < 9; ++a) s0b += s->f[IDX(p, a, j, i)];
      node_inputs(s, w.in, w.jn, f, g, h); /* n is never a wall node */
      orc_node_macros(p, w.jn, s->t, f, g, h, m);
      double uzw = w.free ? 0.0 : w.uz, urw = w.free ? m[2] : w.ur;
      double uthw = w.free ? m[3] : w.omega * r_of(p, j);
      if (is_axis_row(p, j)) uthw = 0.0;
      double Tw = (w.thermal && !w.free) ? w.T : m[4];
      /* the equilibrium of the f^ variables is f_eq - S/2 (seeding), so that
       * Eqs. (16)-(17) at b return exactly (rho_n, u_w) */
      /* sum of f_eq - S/2 is rho (1 + u_r / 2r) (sum of Eq. 12) */
      mb[0] = s0b / (1.0 + 0.5 * urw * inv_r(p, j));
      mb[1] = uzw; mb[2] = urw; mb[3] = uthw; mb[4] = Tw;
      orc_feq9(mb[0], mb[1], mb[2], e1);
      orc_node_source(p, j, s->t, mb, e1, S1);
      orc_feq9(m[0], m[1], m[2], e2);
      orc_node_source(p, w.jn, s->t, m, e2, S2);
      int radial = w.jn != j && w.in == i; /* on a radial wall, not a z-end */
      if (p->zou_he && radial) {
        zou_he_f(s, i, j, mb);
      } else {
        for (int a = 0; a < 9; ++a)
          s->f[IDX(p, a, j, i)] = f[a] + (e1[a] - 0.5 * S1[a]) - (e2[a] - 0.5 * S2[a]);
      }
      if (p->swirl) {
        double q1[4], q2[4];
        orc_geq4(p->rho0, uthw, uzw, urw, q1);
        orc_geq4(p->rho0, m[3], m[1], m[2], q2);
        for (int a = 0; a < 4; ++a) s->g[IDX(p, a, j, i)] = g[a] + q1[a] - q2[a];
      }
      if (p->thermal) {
        double q1[4], q2[4];
        orc_heq4(Tw, uzw, urw, q1);
        orc_heq4(m[4], m[1], m[2], q2);
        for (int a = 0; a < 4; ++a) s->h[IDX(p, a, j, i)] = h[a] + q1[a] - q2[a];
      }
    }
}

void orc_step(orc_state* s, int64_t n) {
  const orc_params* p = &s->p;
  for (int64_t k = 0; k < n; ++k) {
#pragma omp parallel for schedule(static) if (par_ok(p))
    for (int j = 0; j < p->nr; ++j)
      for (int i = 0; i < p->nz; ++i) {
        double f[9], g[4], h[4], fo[9], go[4], ho[4], m[5];
        size_t q = (size_t)j * p->nz + i;
        node_inputs(s, i, j, f, g, h);
        if (p->original) {
          /* D lags one level: the velocity of the previous collision */
          double Dr, Dz;
          grad_terms(p, s->uzp, s->urp, i, j, &Dr, &Dz);
          orc_node_collide_orig(p, j, s->t, f, Dr, Dz, fo, m);
          s->uzn[q] = m[1];
          s->urn[q] = m[2];
        } else {
          orc_node_collide(p, j, s->t, f, g, h, fo, go, ho, m);
        }
        for (int a = 0; a < 9; ++a) s->fs[IDX(p, a, j, i)] = fo[a];
        if (p->swirl)
          for (int a = 0; a < 4; ++a) s->gs[IDX(p, a, j, i)] = go[a];
        if (p->thermal)
          for (int a = 0; a < 4; ++a) s->hs[IDX(p, a, j, i)] = ho[a];
        s->spd[q] = sqrt(m[1] * m[1] + m[2] * m[2]);
      }
    if (p->original) {
      double* tz = s->uzp; s->uzp = s->uzn; s->uzn = tz;
      double* tr = s->urp; s->urp = s->urn; s->urn = tr;
    }
    s->have_spd = 1;
    stream_all(s);
    s->t += 1;
    wet_substitute(s);
  }
}

/* Eq. (57): max over nodes of | |u|(t) - |u|(t-1) |, t the current level.
 * Returns NaN when any node holds a NaN, and -1 when no previous level is
 * known (no step taken since seeding or loading). */
double orc_residual(const orc_state* s) {
  const orc_params* p = &s->p;
  if (!s->have_spd) return -1.0;
  double res = 0.0;
  int bad = 0;
  for (int j = 0; j < p->nr; ++j)
    for (int i = 0; i < p->nz; ++i) {
      double m[5];
      state_macros(s, i, j, m);
      double d = fabs(sqrt(m[1] * m[1] + m[2] * m[2]) -
                      s->spd[(size_t)j * p->nz + i]);
      if (d != d) bad = 1;
      else if (d > res) res = d;
    }
  return bad ? NAN : res;
}

/* Raw state access for the tests (pre-collision f^, g, h at time t). */
void orc_get_state(const orc_state* s, double* f, double* g, double* h) {
  size_t n = nodes(&s->p);
  if (f) memcpy(f, s->f, 9 * n * sizeof(double));
  if (g) memcpy(g, s->g, 4 * n * sizeof(double));
  if (h) memcpy(h, s->h, 4 * n * sizeof(double));
}

void orc_set_state(orc_state* s, const double* f, const double* g,
                   const double* h, int64_t t) {
  size_t n = nodes(&s->p);
  if (f) memcpy(s->f, f, 9 * n * sizeof(double));
  if (g) memcpy(s->g, g, 4 * n * sizeof(double));
  if (h) memcpy(s->h, h, 4 * n * sizeof(double));
  s->t = t;
  s->have_spd = 0;
}

/* Streaming alone, exposed for the permutation tests: state <- stream(in). */
void orc_stream_only(orc_state* s, const double* fs, const double* gs,
                     const double* hs) {
  size_t n = nodes(&s->p);
  memcpy(s->fs, fs, 9 * n * sizeof(double));
  if (gs) memcpy(s->gs, gs, 4 * n * sizeof(double));
  if (hs) memcpy(s->hs, hs, 4 * n * sizeof(double));
  stream_all(s);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Layout probe for the ctypes mirror of orc_params. */
size_t orc_sizeof_params(void) { return sizeof(orc_params); }
