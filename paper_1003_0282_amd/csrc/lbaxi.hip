// lbaxi.hip -- kernels and host runtime behind include/lbaxi.h.
//
// One fused kernel advances every lattice of a handle by one time step:
// each thread owns one node, pulls its 9 (+4 +4) populations from the
// post-collision buffer of the previous step applying the boundary rules,
// computes the macros of Eqs. (16)-(17), collides f with Eqs. (12)-(13) (or
// the MRT model of Sec. III B, or, for comparison, the original scheme of
// Sec. II) and g, h with Eqs. (53)-(54), and writes its populations to the
// other buffer at its own address.  Wet-node walls are rebuilt by a second
// kernel and ghost slots filled by a third.  Work is described by a tile
// table {instance, z0, r0} so that hundreds of uneven lattices share one
// (optionally persistent) launch; runs are replayed from HIP graphs of K
// steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbaxi.h"
#include "lbaxi_device.hpp"

using namespace lbx;

// ============================================================================
// kernels
// ============================================================================

struct Tile {
  int inst, z0, r0, pad;
};

struct TileRange {
  int start, end, stride;
};

// Tiles handled by this workgroup.  With xcd_aware the grid is split into 8
// interleaved groups (workgroup b runs on XCD b % 8), each walking its own
// contiguous band of tiles so that neighbouring tiles share one L2.
__device__ inline TileRange tile_range(int ntiles, int xcd) {
  TileRange t;
  const int G = gridDim.x, b = blockIdx.x;
  if (xcd && G >= 8 && (G & 7) == 0) {
    const int x = b & 7, q = G >> 3;
    t.start = (int)((long long)ntiles * x / 8) + (b >> 3);
    t.end = (int)((long long)ntiles * (x + 1) / 8);
    t.stride = q;
  } else {
    t.start = b;
    t.end = ntiles;
    t.stride = G;
  }
  return t;
}

// S: storage type of populations and fields; R: compute type.
template <typename S>
struct StepArgs {
  const InstP* ip;
  const Tile* tiles;
  const int* ntiles;
  const S* src;
  S* dst;
  double* spd;            // |u| of the level processed (Eq. 57), always FP64
  const long long* tdev;  // time base in device memory (graph replays) or NULL
  long long t0;           // time level when tdev is NULL
  int k;                  // step index inside a graph
  int mode;               // MODE_PRE | MODE_SPEED
  int tzlog;              // log2 of tile_z
  int tr;
  int xcd;
  int nt_store;
  // original scheme: lagged velocity fields (u_z at +0, u_r at +lag_stride,
  // packed [nr][nz] per lattice at its field offset), read and written
  const S* lag_src;
  S* lag_dst;
  long long lag_stride;
};

// The two lagged velocity buffers of the original scheme, for the macro and
// residual kernels (the one of parity D.cur holds the last collided level).
struct Lag {
  const void* A;
  const void* B;
  long long stride;
};

template <typename S>
__device__ inline void st(S* p, S v, int nt) {
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Pull of one node (i, j) into registers; on an axis row the swirl
// populations are replaced by the non-equilibrium extrapolation of row 1
// (Sec. IV B), computed before the node's own pull so that the two
// population sets are never live together.
// Swirl populations of axis node (i, 0): the non-equilibrium part of row 1
// (Sec. IV B), g(i,0) = g(i,1) - g_eq(i,1) with row 1's macros, taken at the
// storage precision like every population the step reads.
template <typename S, typename R, int F>
__device__ inline void axis_swirl(const InstP& P, const PR<R>& p, const S* s, int i, bool pre,
                                  R* gn) {
  R f1[9], g1[4], h1[4];
  load_node<S, R, F>(P, s, i, 1, pre, f1, g1, h1);
  const Mac<R> m1 = macros<R, F>(p, make_row<R, F>(p, 1), false, f1, g1, h1);
  const R q = (R)0.25 * p.rho0 * m1.uth;
#pragma unroll
  for (int a = 0; a < 4; ++a)
    gn[a] = (R)(S)(g1[a] - q * ((R)1 + (R)2 * ((R)ez4(a) * m1.uz + (R)er4(a) * m1.ur)));
}

template <typename S, typename R, int F>
__device__ inline void pull_plain(const InstP& P, const PR<R>& p, const S* s, int i, int j,
                                  bool pre, R* f, R* g, R* h, bool axis_g = true) {
  const bool axis_row = axis_g && (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  R gn[4];
  if ((F & F_SWIRL) && axis_row) axis_swirl<S, R, F>(P, p, s, i, pre, gn);
  load_node<S, R, F>(P, s, i, j, pre, f, g, h);
  if ((F & F_SWIRL) && axis_row) {
#pragma unroll
    for (int a = 0; a < 4; ++a) g[a] = gn[a];
  }
}

// ---- wet-node walls ------------------------------------------------------------
// The paper treats the walls of its rotating flows by non-equilibrium
// extrapolation (Sec. IV B, its Ref. 59).  With LBAXI_WET_WALLS the wall runs
// through the outermost node row / column of every wall side; after each
// streaming step the state of a wall node b is rebuilt from its inner
// neighbour n:
//   f^(b) = E(rho_b, u_w; b) + [f^(n) - E(rho_n, u_n; n)],  E = f_eq - S/2,
//   g(b)  = g_eq(rho0 u_th,w, u_w) + [g(n) - g_eq(n)],  h likewise with T_w,
// (rho_n, u_n) being n's macros (Eqs. 16-17), E the equilibrium of the f^
// variables (Eqs. 6, 12 with the wall values at b), and rho_b chosen so that
// b keeps the mass it streamed in (its links out of the domain bounce back):
// sum E(rho, u) = rho (1 + u_r / 2r).  A node on a z-end and a radial wall
// takes the z-end's values and its diagonal inner neighbour; a free-slip
// segment is a wet node with u_w = (0, u_r,n), u_th,n and T_n.  Wall nodes
// keep their own g on the axis row.
struct WetRule {
  int in, jn, free_, thermal;
  double uz, ur, omega, T;
};

// The side of a wall node is chosen at run time; its parameters are read
// from the lattice's parameter block in memory (Pg) rather than from the
// register copy P, which a runtime member choice would push to scratch.
__device__ inline bool wet_rule(const InstP& P, const InstP* Pg, int i, int j, WetRule* w) {
  if (!P.wet) return false;
  const bool west = i == 0 && P.side[WEST].kind != SIDE_PERIODIC;
  const bool east = !west && i == P.nz - 1 && P.side[EAST].kind != SIDE_PERIODIC;
  const bool north = j == P.nr - 1 && P.side[NORTH].kind == SIDE_WALL;
  const bool south = j == 0 && P.side[SOUTH].kind == SIDE_WALL;
  if (!west && !east && !north && !south) return false;
  if (!w) return true;
  w->in = i + (west ? 1 : (east ? -1 : 0));
  w->jn = j + (north ? -1 : (south ? 1 : 0));
  const int side = west ? WEST : (east ? EAST : (north ? NORTH : SOUTH));
  const SideP* Q = &Pg->side[side];
  if (west || east) {
    int kind;
    zseg_g(P, Q, j, kind, w->omega, w->thermal, w->T);
    w->free_ = kind == SIDE_FREESLIP;
  } else {
    w->free_ = 0;
    w->omega = cload(&Q->omega);
    w->thermal = cload(&Q->thermal);
    w->T = cload(&Q->T);
  }
  w->uz = cload(&Q->uz);
  w->ur = cload(&Q->ur);
  return true;
}

// Source of direction a in velocity space with P = 3 e.u + 4.5 (e.u)^2 -
// 1.5 u^2: Eq. (12), S = w (1 + P) [3 (e - u).F - rho u_r / r], or for the
// MRT model S = M^-1 S~ = w [3 (e - u).F + 9 (e.u)(e.F)] - (u_r / r) f_eq,
// the velocity-space form of Eq. (51) plus the mass source.
template <typename R, int F>
__device__ inline R src_a(int a, R rho, R uz, R ur, R Fz, R Fr, R ir, R Pa) {
  const R ez = (R)ez9(a), er = (R)er9(a), w = (R)w9(a);
  const R eF3 = (R)3 * ((ez - uz) * Fz + (er - ur) * Fr);
  if (F & F_MRT)
    return w * (eF3 + (R)9 * (ez * uz + er * ur) * (ez * Fz + er * Fr)) -
           w * rho * ((R)1 + Pa) * ur * ir;
  return w * ((R)1 + Pa) * (eF3 - rho * ur * ir);
}

// E_a = f_eq - S/2 of direction a in deviation form (f_eq = w (drho + rho P)).
template <typename R, int F>
__device__ inline R eq_hat(int a, R drho, R rho, R uz, R ur, R Fz, R Fr, R ir) {
  const R ez = (R)ez9(a), er = (R)er9(a), w = (R)w9(a);
  const R eu = ez * uz + er * ur;
  const R Pa = (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * (uz * uz + ur * ur);
  return w * (drho + rho * Pa) - (R)0.5 * src_a<R, F>(a, rho, uz, ur, Fz, Fr, ir, Pa);
}

// Zou-He no-slip at a node on a radial wall (the paper's Ref. 47), f only:
// the populations that streamed in from the fluid side (in f) are kept; the
// three with e_r = SGN (coming from beyond the wall) follow from Eqs.
// (16)-(17) at the wall velocity (u_z,w, 0): sum e_r f = -G_r / 2 and
// sum e_z f = u_z,w sum f - G_z / 2, from non-equilibrium bounce-back along
// the normal, f_n - E_n = f_m - E_m, and from an equal share of the rest
// between the two diagonals.  In deviation form the w rho0 parts cancel
// except in the mass, rho = sum f.
template <typename R, int F, int SGN>
__device__ inline void zou_he(const PR<R>& p, const Row<R>& rb, R uzw, R Gz, R Gr, R* f) {
  const R* fo = f;  // the known populations; only the unknown slots are written
  constexpr int N = SGN > 0 ? 2 : 4, M = SGN > 0 ? 4 : 2;  // normal pair
  constexpr int DP = SGN > 0 ? 5 : 8, DM = SGN > 0 ? 6 : 7;  // e_z = +1 / -1 unknowns
  constexpr int KP = SGN > 0 ? 8 : 5, KM = SGN > 0 ? 7 : 6;  // e_z = +1 / -1 knowns
  const R D0 = fo[0] + (fo[1] + fo[3]);
  const R Dk = fo[M] + (fo[KP] + fo[KM]);
  const R Ud = Dk - (R)SGN * (R)0.5 * Gr;
  const R drho = D0 + Dk + Ud;
  const R rho = p.rho0 + drho;
  const R Zk = (fo[1] - fo[3]) + (fo[KP] - fo[KM]);
  const R Dz = uzw * rho - (R)0.5 * Gz - Zk;
  const R dn = fo[M] + eq_hat<R, F>(N, drho, rho, uzw, (R)0, Gz, Gr, rb.ir) -
               eq_hat<R, F>(M, drho, rho, uzw, (R)0, Gz, Gr, rb.ir);
  f[N] = dn;
  f[DP] = (R)0.5 * (Ud - dn + Dz);
  f[DM] = (R)0.5 * (Ud - dn - Dz);
}

template <typename S, typename R, int F>
__device__ inline void wall_state(const InstP& P, const PR<R>& p, const S* s, int i, int j,
                                  const WetRule& w, R* f, R* g, R* h) {
  R s0d;
  {
    R fo[9], go[4], ho[4];
    load_node<S, R, F>(P, s, i, j, false, fo, go, ho);
    s0d = ((fo[0] + fo[1]) + (fo[2] + fo[3])) + ((fo[4] + fo[5]) + (fo[6] + fo[7])) + fo[8];
  }
  R fn[9], gn[4], hn[4];
  pull_plain<S, R, F>(P, p, s, w.in, w.jn, false, fn, gn, hn);
  const bool axis_n = (w.jn == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  const bool axis_b = (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  const Row<R> rn = make_row<R, F>(p, w.jn);
  const Row<R> rb = make_row<R, F>(p, j);
  const Mac<R> m = macros<R, F>(p, rn, axis_n, fn, gn, hn);
  const R uzw = w.free_ ? (R)0 : (R)w.uz;
  const R urw = w.free_ ? m.ur : (R)w.ur;
  R uthw = w.free_ ? m.uth : (R)(w.omega * (P.r0 + (double)j));
  if (axis_b) uthw = (R)0;
  const R dTw = (w.thermal && !w.free_) ? (R)(w.T - P.T_ref) : m.dT;
  const R x = (R)0.5 * urw * rb.ir;
  const R drhob = (s0d - p.rho0 * x) * rcp((R)1 + x);
  const R rhob = p.rho0 + drhob;
  R Fzb = p.a_t;
  if (F & F_THERMAL) Fzb += p.rho0 * p.gbeta * dTw;
  R Frb = -(R)2 * p.mu0 * urw * rb.ir2;
  if (F & F_SWIRL) Frb += p.rho0 * uthw * uthw * rb.ir;
  const bool zou = P.zou && w.in == i && w.jn != j;  // Zou-He on a radial wall
  if (zou) {
    // corners and z-ends keep the extrapolation, g and h too; the node's own
    // streamed-in populations are loaded into f and completed in place
    R gd[4], hd[4];
    load_node<S, R, F>(P, s, i, j, false, f, gd, hd);
    const R Gr = (F & F_SWIRL) ? p.rho0 * uthw * uthw * rb.ir : (R)0;
    if (w.jn < j)
      zou_he<R, F, -1>(p, rb, uzw, Fzb, Gr, f);
    else
      zou_he<R, F, 1>(p, rb, uzw, Fzb, Gr, f);
  } else {
#pragma unroll
    for (int a = 0; a < 9; ++a)
      f[a] = fn[a] + eq_hat<R, F>(a, drhob, rhob, uzw, urw, Fzb, Frb, rb.ir) -
             eq_hat<R, F>(a, m.drho, m.rho, m.uz, m.ur, m.Fz, m.Fr, rn.ir);
  }
  if (F & F_SWIRL) {
    const R qb = (R)0.25 * p.rho0 * uthw, qn = (R)0.25 * p.rho0 * m.uth;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const R ez = (R)ez4(a), er = (R)er4(a);
      g[a] = gn[a] + qb * ((R)1 + (R)2 * (ez * uzw + er * urw)) -
             qn * ((R)1 + (R)2 * (ez * m.uz + er * m.ur));
    }
  }
  if (F & F_THERMAL) {
    const R Tb = p.T_ref + dTw, Tn = p.T_ref + m.dT;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const R ez = (R)ez4(a), er = (R)er4(a);
      h[a] = hn[a] + (R)0.25 * (Tb * ((R)1 + (R)2 * (ez * uzw + er * urw)) -
                                Tn * ((R)1 + (R)2 * (ez * m.uz + er * m.ur)));
    }
  }
}

// A value that is the same on every active lane, moved to scalar registers
// (the step kernel's waves never straddle a row, so the row constants are
// wave-uniform; held in SGPRs they cost no VGPRs).
__device__ inline double uni(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ inline float uni(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(unsigned, x)));
}
template <typename R, int F>
__device__ inline Row<R> uni_row(Row<R> w) {
  w.ir = uni(w.ir);
  w.ir2 = uni(w.ir2);
  if (F & F_MRT) {
    w.gam = uni(w.gam);
  } else {
    w.omp = uni(w.omp);
    w.omm = uni(w.omm);
    w.c0 = uni(w.c0);
    w.cp = uni(w.cp);
    w.cm = uni(w.cm);
  }
  if (F & F_SWIRL) {
    w.gp = uni(w.gp);
    w.gm = uni(w.gm);
    w.gsk = uni(w.gsk);
  }
  if (F & F_THERMAL) {
    w.hp = uni(w.hp);
    w.hm = uni(w.hm);
  }
  return w;
}

// Macros, collision and store of one pulled node.  uniform_row: j is the
// same on every lane of the wave; stored: f, g, h hold the values as loaded
// from storage (not a rebuilt wall node).  The swirl and temperature
// populations are
// collided and stored before f is collided, so that they are not live
// through the f collision.
template <typename S, typename R, int F>
__device__ inline void finish_node(const StepArgs<S>& A, const InstP& P, const PR<R>& p, int i,
                                   int j, R* f, R* g, R* h, bool uniform_row = false,
                                   bool stored = false) {
  const bool axis_row = (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  const Row<R> rw = uniform_row ? uni_row<R, F>(make_row<R, F>(p, __builtin_amdgcn_readfirstlane(j)))
                                : make_row<R, F>(p, j);
  Mac<R> m;
  if (F & F_ORIG) {
    R Dr, Dz;
    const S* lz = A.lag_src + P.off_fld;
    lag_grad<S, R>(P, rw, lz, lz + A.lag_stride, i, j, Dr, Dz);
    m = macros_orig<R>(p, rw, f, Dr, Dz);
    collide_f_orig<R>(p, rw, m, f);
    S* ld = A.lag_dst + P.off_fld + (long long)j * P.nz + i;
    ld[0] = (S)m.uz;
    ld[A.lag_stride] = (S)m.ur;
  } else if (sizeof(S) < sizeof(R) && stored) {
    // float storage, populations as loaded: only the floats stay live
    // across the macros.  The empty asm makes each float opaque to the
    // compiler, so the collision converts it again instead of keeping the
    // double (2 VGPRs) alive.
    float fl[9], gl[4], hl[4];
    R fa[9], ga[4], ha[4];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      fl[a] = (float)f[a];
      asm volatile("" : "+v"(fl[a]));
      fa[a] = (R)fl[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (F & F_SWIRL) {
        gl[a] = (float)g[a];
        asm volatile("" : "+v"(gl[a]));
        ga[a] = (R)gl[a];
      }
      if (F & F_THERMAL) {
        hl[a] = (float)h[a];
        asm volatile("" : "+v"(hl[a]));
        ha[a] = (R)hl[a];
      }
    }
    m = macros<R, F>(p, rw, axis_row, fa, ga, ha);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      asm volatile("" : "+v"(fl[a]));
      f[a] = (R)fl[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (F & F_SWIRL) {
        asm volatile("" : "+v"(gl[a]));
        g[a] = (R)gl[a];
      }
      if (F & F_THERMAL) {
        asm volatile("" : "+v"(hl[a]));
        h[a] = (R)hl[a];
      }
    }
  } else {
    m = macros<R, F>(p, rw, axis_row, f, g, h);
  }
  S* d = A.dst + P.off;
  const int pl = P.plane;
  const unsigned ob = (unsigned)nidx(P, j, i) * (unsigned)sizeof(S);
  if (!(F & F_ORIG)) {
    collide<R, F>(p, rw, m, f, g, h, 2);
    if (F & F_SWIRL) {
#pragma unroll
      for (int a = 0; a < 4; ++a) st(ptrb(d + (9 + a) * pl, ob), (S)g[a], A.nt_store);
    }
    if (F & F_THERMAL) {
      const int hb = (F & F_SWIRL) ? 13 : 9;
#pragma unroll
      for (int a = 0; a < 4; ++a) st(ptrb(d + (hb + a) * pl, ob), (S)h[a], A.nt_store);
    }
    collide<R, F>(p, rw, m, f, g, h, 1);
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) st(ptrb(d + a * pl, ob), (S)f[a], A.nt_store);
  if ((F & F_ORIG) && (F & F_SWIRL)) {
#pragma unroll
    for (int a = 0; a < 4; ++a) st(ptrb(d + (9 + a) * pl, ob), (S)g[a], A.nt_store);
  }
  if ((F & F_ORIG) && (F & F_THERMAL)) {
    const int hb = (F & F_SWIRL) ? 13 : 9;
#pragma unroll
    for (int a = 0; a < 4; ++a) st(ptrb(d + (hb + a) * pl, ob), (S)h[a], A.nt_store);
  }
  if (A.mode & MODE_SPEED)
    A.spd[P.off_fld + (long long)j * P.nz + i] = (double)sqrt(m.uz * m.uz + m.ur * m.ur);
}

// Boundary node number p of a lattice: row 0, row nr-1, then columns 0 and
// nz-1 without their corners.
__device__ inline void perimeter_node(const InstP& P, int p, int& i, int& j) {
  const int nz = P.nz, nr = P.nr;
  if (p < nz) { i = p; j = 0; return; }
  p -= nz;
  if (p < nz) { i = p; j = nr - 1; return; }
  p -= nz;
  if (p < nr - 2) { i = 0; j = 1 + p; return; }
  p -= nr - 2;
  i = nz - 1; j = 1 + p;
}

// Waves per SIMD the step kernel is compiled for: five (at most 96 VGPRs)
// where the field set fits without spilling, four (128) for swirl together
// with temperature or with MRT, three (168) for the wet-wall instance.
constexpr int step_waves(int F) {
  return (F & F_WETZ) ? 3 : ((F & F_SWIRL) && (F & (F_THERMAL | F_MRT))) ? 4 : 5;
}

__device__ inline bool radial_wall_row(const InstP& P, int j) {
  return (j == P.nr - 1 && P.side[NORTH].kind == SIDE_WALL) ||
         (j == 0 && P.side[SOUTH].kind == SIDE_WALL);
}

// Largest workgroup of the step kernel: 512 threads where the z-end wall
// rebuild is inlined (it needs up to 168 VGPRs at three waves per SIMD).
constexpr int step_block_max(int F) { return (F & F_WETZ) ? 512 : 1024; }

// One node (i, j) of a step tile: pull (or, for a wet z-end wall node, the
// rebuild), macros, collision, store.
template <typename S, typename R, int F>
__device__ __forceinline__ void step_node(const StepArgs<S>& A, const Tile& T, const InstP& P,
                                          long long t, bool pre, int i, int j) {
  // wet wall nodes (only in the F_WETZ instance, which every handle with
  // wet-node walls uses) are rebuilt after the pull, the z-end ones here
  // and those of the radial wall rows by k_wall, except on the first step
  // after seeding, where they collide their seeded state like any node
  constexpr int FB = F & ~F_WETZ;
  const bool wall = (F & F_WETZ) && P.wet && wet_rule(P, nullptr, i, j, nullptr);
  const bool rebuild = wall && !pre;
  if (rebuild && radial_wall_row(P, j)) return;
  const PR<R> p = make_pr<R>(P, t);
  R f[9], g[4], h[4];
  if ((F & F_WETZ) && rebuild) {
    WetRule w;
    wet_rule(P, A.ip + T.inst, i, j, &w);
    wall_state<S, R, FB>(P, p, A.src + P.off, i, j, w, f, g, h);
  } else {
    pull_plain<S, R, FB>(P, p, A.src + P.off, i, j, pre, f, g, h, !wall);
  }
  finish_node<S, R, FB>(A, P, p, i, j, f, g, h, true, !(F & F_WETZ));
}

// One time step: pull (padded rows, no boundary tests), macros, collision,
// store at the node's own slots of the other buffer.  The halo kernel then
// completes the boundary rules for the next pull.  F_WETZ (handles with
// wet-node walls): the z-end wall nodes of rows that also hold fluid nodes
// are rebuilt here, by their own lanes, from the inner neighbour that the
// same wave has just pulled (its lines are in the cache), so that the wall
// kernel is left only the radial wall rows and every row off them is
// written whole by this kernel.
template <typename S, typename R, int F>
__global__ void __launch_bounds__(step_block_max(F))
    __attribute__((amdgpu_waves_per_eu(step_waves(F)))) k_step(StepArgs<S> A) {
  const long long t = A.tdev ? (*A.tdev + A.k) : A.t0;
  const int ntiles = *A.ntiles;
  const TileRange tr = tile_range(ntiles, A.xcd);
  const int tz = 1 << A.tzlog;
  const int li = threadIdx.x & (tz - 1), lj = threadIdx.x >> A.tzlog;
  const bool pre = A.mode & MODE_PRE;
  for (int ti = tr.start; ti < tr.end; ti += tr.stride) {
    const Tile T = cload(A.tiles + ti);
    const InstP P = cload(A.ip + T.inst);
    const int i = T.z0 + li, j = T.r0 + lj;
    if (i >= P.nz || j >= P.nr) continue;
    // the body of step_node, written out: called from here, that function
    // compiled to a different (longer) instruction schedule of this loop
    constexpr int FB = F & ~F_WETZ;
    const bool wall = (F & F_WETZ) && P.wet && wet_rule(P, nullptr, i, j, nullptr);
    const bool rebuild = wall && !pre;
    if (rebuild && radial_wall_row(P, j)) continue;
    const PR<R> p = make_pr<R>(P, t);
    R f[9], g[4], h[4];
    if ((F & F_WETZ) && rebuild) {
      WetRule w;
      wet_rule(P, A.ip + T.inst, i, j, &w);
      wall_state<S, R, FB>(P, p, A.src + P.off, i, j, w, f, g, h);
    } else {
      pull_plain<S, R, FB>(P, p, A.src + P.off, i, j, pre, f, g, h, !wall);
    }
    finish_node<S, R, FB>(A, P, p, i, j, f, g, h, true, !(F & F_WETZ));
  }
}

// Wet wall nodes of every running lattice after a streaming step (one
// thread per perimeter node, tiles of the halo list): rebuild from the inner
// neighbour, then macros, collision and store like k_step.  Reads the same
// source buffer as k_step and writes other nodes of the same destination.
template <typename S, typename R, int F>
__device__ __forceinline__ void wall_node(const StepArgs<S>& A, const Tile& T, const InstP& P,
                                          int q) {
  if (q >= 2 * P.nz + 2 * (P.nr - 2)) return;
  int i, j;
  perimeter_node(P, q, i, j);
  // with MODE_WETZ the step kernel has rebuilt every wall node off the
  // radial wall rows
  if ((A.mode & MODE_WETZ) && !radial_wall_row(P, j)) return;
  WetRule w;
  if (!wet_rule(P, A.ip + T.inst, i, j, &w)) return;
  const long long t = A.tdev ? (*A.tdev + A.k) : A.t0;
  const PR<R> p = make_pr<R>(P, t);
  R f[9], g[4], h[4];
  wall_state<S, R, F>(P, p, A.src + P.off, i, j, w, f, g, h);
  finish_node<S, R, F>(A, P, p, i, j, f, g, h);
}

template <typename S, typename R, int F>
__global__ void __launch_bounds__(256) k_wall(StepArgs<S> A) {
  const int ti = blockIdx.x;
  if (ti >= *A.ntiles) return;
  const Tile T = cload(A.tiles + ti);
  const InstP P = cload(A.ip + T.inst);
  if (!P.wet) return;
  wall_node<S, R, F>(A, T, P, T.z0 + threadIdx.x);
}

// Ghost-slot fill after a step: tiles here are {instance, first perimeter
// node, 0, 0}, one thread per perimeter node.
template <typename S, int F>
__device__ __forceinline__ void halo_node(const InstP* ip, const Tile& T, const InstP& P, S* buf,
                                          int p) {
  if (p >= 2 * P.nz + 2 * (P.nr - 2)) return;
  int i, j;
  perimeter_node(P, p, i, j);
  halo_fill<S, F>(P, ip + T.inst, buf + P.off, i, j);
}

template <typename S, int F>
__global__ void __launch_bounds__(256) k_halo(const InstP* ip, const Tile* tiles,
                                              const int* ntiles, S* buf) {
  const int ti = blockIdx.x;
  if (ti >= *ntiles) return;
  const Tile T = cload(tiles + ti);
  const InstP P = cload(ip + T.inst);
  halo_node<S, F>(ip, T, P, buf, T.z0 + threadIdx.x);
}

// The wall part of a step taken in the step's own launch.
struct WallPart {
  const Tile* htiles;  // perimeter tiles of the running lattices
  const int* nh;       // their count
  int ns;              // workgroups of the step part (one per tile of the step's list)
};

// Step and wet-wall work of a time step in one launch, for handles with
// wet-node walls and few lattices, where each kernel of a step is a short
// chain of dependent loads and the step costs about the sum of its kernels.
// Workgroups [0, ns) do what k_step does for one tile each, the others what
// k_wall does for one perimeter tile each: both read only the source buffer
// and write disjoint nodes of the destination, so the two parts need no
// order between them.  The ghost slots are filled by k_halo afterwards, as
// after the separate kernels.  Same arithmetic per node.
template <typename S, typename R, int F>
__global__ void __launch_bounds__(step_block_max(F)) k_step_wall(StepArgs<S> A, WallPart B) {
  constexpr int FB = F & ~F_WETZ;
  const int b = blockIdx.x;
  if (b < B.ns) {
    if (b >= *A.ntiles) return;
    const long long t = A.tdev ? (*A.tdev + A.k) : A.t0;
    const Tile T = cload(A.tiles + b);
    const InstP P = cload(A.ip + T.inst);
    const int tz = 1 << A.tzlog;
    const int i = T.z0 + (threadIdx.x & (tz - 1)), j = T.r0 + (threadIdx.x >> A.tzlog);
    if (i < P.nz && j < P.nr) step_node<S, R, F>(A, T, P, t, A.mode & MODE_PRE, i, j);
  } else {
    const int w = b - B.ns;
    if (w >= *B.nh) return;
    const Tile T = cload(B.htiles + w);
    const InstP P = cload(A.ip + T.inst);
    if (!P.wet) return;
    for (int q = threadIdx.x; q < 256; q += blockDim.x) wall_node<S, R, FB>(A, T, P, T.z0 + q);
  }
}

// Equilibrium seeding: f^ = f_eq - S/2 (S of the collision model), g = g_eq,
// h = h_eq.
template <typename S, typename R, int F>
__global__ void __launch_bounds__(1024) k_seed(const InstP* ip, const Tile* tiles,
                                               const int* ntiles, S* buf, const S* rho_in,
                                               const S* uz_in,
                                               const S* ur_in, const S* uth_in, const S* T_in,
                                               int tzlog, const S* lag, long long lag_stride) {
  const int ti = blockIdx.x;
  if (ti >= *ntiles) return;
  const Tile T = cload(tiles + ti);
  const InstP P = cload(ip + T.inst);
  const int tz = 1 << tzlog;
  const int i = T.z0 + (threadIdx.x & (tz - 1)), j = T.r0 + (threadIdx.x >> tzlog);
  if (i >= P.nz || j >= P.nr) return;
  const PR<R> p = make_pr<R>(P, 0);
  const long long fo = P.off_fld + (long long)j * P.nz + i;
  const bool axis_row = (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  const R uz = uz_in ? (R)uz_in[fo] : (R)0;
  const R ur = (ur_in && !axis_row) ? (R)ur_in[fo] : (R)0;
  const R uth = ((F & F_SWIRL) && uth_in && !axis_row) ? (R)uth_in[fo] : (R)0;
  const R dT = ((F & F_THERMAL) && T_in) ? (R)T_in[fo] - p.T_ref : (R)0;
  const R drho = rho_in ? (R)rho_in[fo] - p.rho0 : (R)0;
  const R rho = p.rho0 + drho;
  const R ir = make_row<R, F>(p, j).ir;
  R Fz = p.a_t;
  if (F & F_THERMAL) Fz += p.rho0 * p.gbeta * dT;
  R Fr = -(R)2 * p.mu0 * ur * ir * ir;
  if (F & F_SWIRL) Fr += p.rho0 * uth * uth * ir;
  const R usq = uz * uz + ur * ur;
  S* d = buf + P.off;
  const int pl = P.plane, o = nidx(P, j, i);
  if (F & F_ORIG) {
    // f~ = f_eq - G/2 with G of Eq. (7), D from the seeded velocity field
    // (already in the lagged buffer)
    const Row<R> rw = make_row<R, F>(p, j);
    R Dr, Dz;
    lag_grad<S, R>(P, rw, lag + P.off_fld, lag + P.off_fld + lag_stride, i, j, Dr, Dz);
    const R Fro = p.mu0 * ir * Dr - (R)2 * p.mu0 * ur * rw.ir2 - rho * ur * ur * ir;
    const R Fzo = p.mu0 * ir * Dz - rho * uz * ur * ir + p.a_t;
    const R uF = uz * Fzo + ur * Fro;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const R ez = (R)ez9(a), er = (R)er9(a), wa = (R)w9(a);
      const R eu = ez * uz + er * ur;
      const R Pa = (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * usq;
      const R G = wa * ((R)3 * ((R)1 + Pa) * (ez * Fzo + er * Fro - uF) - rho * ur * ir);
      d[a * pl + o] = (S)(wa * (drho + rho * Pa) - (R)0.5 * G);
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const R ez = (R)ez9(a), er = (R)er9(a), w = (R)w9(a);
    const R eu = ez * uz + er * ur;
    const R Pa = (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * usq;
    const R Sa = src_a<R, F>(a, rho, uz, ur, Fz, Fr, ir, Pa);
    d[a * pl + o] = (S)(w * (drho + rho * Pa) - (R)0.5 * Sa);
  }
  if (F & F_SWIRL) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
      d[(9 + a) * pl + o] =
          (S)((R)0.25 * p.rho0 * uth * ((R)1 + (R)2 * ((R)ez4(a) * uz + (R)er4(a) * ur)));
  }
  if (F & F_THERMAL) {
    const int hb = (F & F_SWIRL) ? 13 : 9;
    const R Tv = p.T_ref + dT;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      d[(hb + a) * pl + o] =
          (S)((R)0.25 * (dT + Tv * (R)2 * ((R)ez4(a) * uz + (R)er4(a) * ur)));
  }
}

// Original scheme: the seeded velocity written to the lagged buffer that the
// first step (and the seeding of f~) takes its gradients from.
template <typename S>
__global__ void __launch_bounds__(1024) k_seed_lag(const InstP* ip, const Tile* tiles,
                                                   const int* ntiles, const S* uz_in,
                                                   const S* ur_in, S* lag, long long lag_stride,
                                                   int tzlog) {
  const int ti = blockIdx.x;
  if (ti >= *ntiles) return;
  const Tile T = cload(tiles + ti);
  const InstP P = cload(ip + T.inst);
  const int tz = 1 << tzlog;
  const int i = T.z0 + (threadIdx.x & (tz - 1)), j = T.r0 + (threadIdx.x >> tzlog);
  if (i >= P.nz || j >= P.nr) return;
  const long long fo = P.off_fld + (long long)j * P.nz + i;
  const bool axis_row = (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  lag[fo] = uz_in ? uz_in[fo] : (S)0;
  lag[fo + lag_stride] = (ur_in && !axis_row) ? ur_in[fo] : (S)0;
}

// Macros at the current level of each lattice (own buffer parity and time).
template <typename S, typename R, int F>
__device__ inline Mac<R> node_macros(const InstP& P, const InstP* Pg, const InstDyn& D,
                                     const S* bufA, const S* bufB, const Lag& lag, int i, int j) {
  const PR<R> p = make_pr<R>(P, D.t);
  const S* s = (D.cur ? bufB : bufA) + P.off;
  R f[9], g[4], h[4];
  if (F & F_ORIG) {
    load_node<S, R, F>(P, s, i, j, D.pre != 0, f, g, h);
    const Row<R> rw = make_row<R, F>(p, j);
    const S* lz = static_cast<const S*>(D.cur ? lag.B : lag.A) + P.off_fld;
    R Dr, Dz;
    lag_grad<S, R>(P, rw, lz, lz + lag.stride, i, j, Dr, Dz);
    return macros_orig<R>(p, rw, f, Dr, Dz);
  }
  WetRule w;
  if (P.wet && !D.pre && wet_rule(P, Pg, i, j, &w))
    wall_state<S, R, F>(P, p, s, i, j, w, f, g, h);
  else
    load_node<S, R, F>(P, s, i, j, D.pre != 0, f, g, h);
  const bool axis_row = (j == 0) && (P.side[SOUTH].kind == SIDE_AXIS);
  // on the axis u_th = 0 and g does not enter the macros of Eqs. (16)-(17)
  return macros<R, F>(p, make_row<R, F>(p, j), axis_row, f, g, h);
}

// Up to 256 threads per workgroup walk the tile's nodes (a tile holds 64 to
// 1024): wet-node wall rebuilds inline here, and workgroups of at most 256
// threads leave them the registers that 1024-thread ones would not.
template <typename S, typename R, int F>
__global__ void __launch_bounds__(256) k_macros(const InstP* ip, const InstDyn* dyn,
                                                const Tile* tiles, const int* ntiles,
                                                const S* bufA, const S* bufB, S* rho, S* uz,
                                                S* ur, S* uth, S* T, int tzlog, int tile_nodes,
                                                Lag lag) {
  const int ti = blockIdx.x;
  if (ti >= *ntiles) return;
  const Tile Tl = cload(tiles + ti);
  const InstP P = cload(ip + Tl.inst);
  const int tz = 1 << tzlog;
#pragma unroll 1
  for (int q = threadIdx.x; q < tile_nodes; q += blockDim.x) {
    const int i = Tl.z0 + (q & (tz - 1)), j = Tl.r0 + (q >> tzlog);
    if (i >= P.nz || j >= P.nr) continue;
    const Mac<R> m = node_macros<S, R, F>(P, ip + Tl.inst, dyn[Tl.inst], bufA, bufB, lag, i, j);
    const long long o = P.off_fld + (long long)j * P.nz + i;
    if (rho) rho[o] = (S)m.rho;
    if (uz) uz[o] = (S)m.uz;
    if (ur) ur[o] = (S)m.ur;
    if (uth) uth[o] = (S)m.uth;
    if (T) T[o] = (S)((R)P.T_ref + m.dT);
  }
}

// Bit pattern of a non-negative double: monotone in the value, and every NaN
// compares above +Inf, so an unsigned max both reduces and flags NaN.
__device__ inline unsigned long long key(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v));
}

// Eq. (57) per lattice: max | |u|(t) - |u|(t-1) | with |u|(t-1) in spd
// (up to 256 threads per workgroup walking the tile, as k_macros).
template <typename S, typename R, int F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) k_residual(const InstP* ip, const InstDyn* dyn,
                                                  const Tile* tiles, const int* ntiles,
                                                  const S* bufA, const S* bufB,
                                                  const double* spd, unsigned long long* res,
                                                  int tzlog, int tile_nodes, Lag lag) {
  __shared__ unsigned long long red[4];
  const int ti = blockIdx.x;
  if (ti >= *ntiles) return;  // uniform per workgroup
  const Tile Tl = cload(tiles + ti);
  const InstP P = cload(ip + Tl.inst);
  const int tz = 1 << tzlog;
  unsigned long long v = 0;
#pragma unroll 1
  for (int q = threadIdx.x; q < tile_nodes; q += blockDim.x) {
    const int i = Tl.z0 + (q & (tz - 1)), j = Tl.r0 + (q >> tzlog);
    if (i >= P.nz || j >= P.nr) continue;
    const Mac<R> m = node_macros<S, R, F>(P, ip + Tl.inst, dyn[Tl.inst], bufA, bufB, lag, i, j);
    const double sp = (double)sqrt(m.uz * m.uz + m.ur * m.ur);
    const unsigned long long k = key(sp - spd[P.off_fld + (long long)j * P.nz + i]);
    v = k > v ? k : v;
  }
  // wave-level max, then across the four waves of the workgroup
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    unsigned long long b = red[0];
    for (int w = 1; w < nw; ++w) b = red[w] > b ? red[w] : b;
    atomicMax(res + Tl.inst, b);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = v;
}

__global__ void k_set_time(long long* t, long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = v;
}

__global__ void k_add_time(long long* t, long long dv) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t += dv;
}

// Plain streaming copy, the bandwidth reference against which the step
// kernel's HBM traffic is calibrated.  A workgroup moves U * 4 KiB: each lane
// issues its U 16-byte loads (coalesced, 4 KiB apart) before the first store,
// so U loads per lane are in flight at once.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int U>
__global__ void __launch_bounds__(256) k_copy(const u32x4* __restrict__ src,
                                              u32x4* __restrict__ dst, long long n) {
  const long long base = (long long)blockIdx.x * (256 * U) + threadIdx.x;
  u32x4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long k = base + 256LL * u;
    if (k < n) v[u] = src[k];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long k = base + 256LL * u;
    if (k < n) __builtin_nontemporal_store(v[u], dst + k);
  }
}

// Residual words of lbaxi_residual_static: a fixed array in device memory
// (one copy per GPU the library runs on, held until the process ends), for
// callers that cannot allocate.  Host code reaches it only through the device
// address hipGetSymbolAddress returns for the current device.
constexpr int STATIC_RESIDUAL_MAX = 8192;  // lattices per handle
static __device__ __align__(256) unsigned long long scratch[STATIC_RESIDUAL_MAX];

// ============================================================================
// host runtime
// ============================================================================

namespace {

thread_local std::string g_err = "no error";

lbaxi_status fail(lbaxi_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LBAXI_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int n_planes(unsigned fields) {
  return 9 + ((fields & LBAXI_SWIRL) ? 4 : 0) + ((fields & LBAXI_THERMAL) ? 4 : 0);
}

size_t elem_size(int prec) { return prec == LBAXI_FP64 ? 8 : 4; }

// Worst-case tile count over the shapes the runtime accepts (tile_z >= 64).
long long max_tiles(const std::vector<lbaxi_desc>& d) {
  long long n = 0;
  for (const auto& x : d) n += (long long)((x.nz + 63) / 64) * x.nr;
  return n;
}

// Boundary nodes of a lattice and the halo workgroups (256 nodes) covering them.
int perimeter(const lbaxi_desc& x) { return 2 * x.nz + 2 * (x.nr - 2); }
long long halo_tiles(const std::vector<lbaxi_desc>& d) {
  long long n = 0;
  for (const auto& x : d) n += (perimeter(x) + 255) / 256;
  return n;
}
// Row-blocked layout of one lattice's populations.  A padded row of one
// population has a 128-byte lead-in (node 0 starts a 128-byte line), nz
// nodes and one spare slot, rounded up to 128 bytes (and to at least the
// length of a ghost-column strip).  The padded rows of all populations for
// one lattice row follow each other (row block), and row blocks follow in
// row order: block 0 holds ghost row -1, block j + 1 node row j, block nr + 1
// ghost row nr.  Two more blocks hold the ghost-column strips of the west
// and the east z-end (rows -1..nr of each population, contiguous).  So the
// plane stride is one padded row and the row stride one row block: the
// populations a wave pulls for a tile lie in three nearby row blocks rather
// than in Q planes a lattice apart.
//
// Plane layout (LBAXI_PLANES, and every lattice whose row blocks would take
// 4 GiB or more): each population's padded rows -1..nr follow each other
// (one plane), then that population's west and east strips; the plane
// stride is a whole plane and the row stride one padded row.  Byte offsets
// then stay inside one population's plane, so such a lattice may hold up to
// 2^31 population elements.  The kernels see only the strides and strip
// offsets and run either layout unchanged.
int row_lead(const lbaxi_desc& x) { return 128 / (x.prec == LBAXI_FP64 ? 8 : 4); }
int strip_len(const lbaxi_desc& x) {
  const int q = row_lead(x);
  return (x.nr + 2 + q - 1) / q * q;
}
int padded_row(const lbaxi_desc& x) {
  const int q = row_lead(x);
  return (q + x.nz + 1 + q - 1) / q * q;
}

struct PopLayout {
  long long plane, pitch, sw, se, total;  // elements (strides, strip offsets, lattice size)
};

PopLayout pop_layout(const lbaxi_desc& x) {
  PopLayout L;
  const long long np = n_planes(x.fields), sl = strip_len(x);
  const long long rb = std::max<long long>(padded_row(x), sl);  // row-block padded row
  const bool planes = (x.fields & LBAXI_PLANES) ||
                      (x.nr + 4) * np * rb * (long long)elem_size(x.prec) >= (1LL << 32);
  if (planes) {
    const long long rp = padded_row(x);
    L.pitch = rp;
    L.sw = (x.nr + 2) * rp;
    L.se = L.sw + sl;
    L.plane = L.sw + 2 * sl;
    L.total = np * L.plane;
  } else {
    L.plane = rb;
    L.pitch = np * rb;
    L.sw = (x.nr + 2) * L.pitch;
    L.se = L.sw + L.pitch;
    L.total = (x.nr + 4) * L.pitch;
  }
  return L;
}
long long lattice_elems(const lbaxi_desc& x) { return pop_layout(x).total; }

// Device workspace: parameters, three work lists (all tiles / tiles of
// running lattices / halo chunks of running lattices) with their counts,
// residual words, the time base, two padded population buffers and |u| of
// Eq. (57).
struct Layout {
  size_t ip, dyn, tiles_all, tiles_run, tiles_halo, counts, res, tdev, bufA, bufB, spd, lagA, lagB,
      total;
  long long lag_stride;  // elements between the u_z and u_r parts of a lagged buffer
  std::vector<long long> off, off_fld;
  long long buf_elems, fld_elems;
};

Layout layout(const std::vector<lbaxi_desc>& d) {
  Layout L;
  const int n = (int)d.size();
  const size_t es = elem_size(d[0].prec);
  const size_t tb = sizeof(Tile) * (size_t)max_tiles(d);
  size_t o = 0;
  L.ip = o; o = align_up(o + sizeof(InstP) * n, 256);
  L.dyn = o; o = align_up(o + sizeof(InstDyn) * n, 256);
  L.tiles_all = o; o = align_up(o + tb, 256);
  L.tiles_run = o; o = align_up(o + tb, 256);
  L.tiles_halo = o; o = align_up(o + sizeof(Tile) * (size_t)halo_tiles(d), 256);
  L.counts = o; o = align_up(o + 4 * sizeof(int), 256);
  L.res = o; o = align_up(o + sizeof(unsigned long long) * n, 256);
  L.tdev = o; o = align_up(o + sizeof(long long), 256);
  long long e = 0, fe = 0;
  for (const auto& x : d) {
    L.off.push_back(e);
    L.off_fld.push_back(fe);
    e += align_up((size_t)lattice_elems(x), 64);
    fe += (long long)x.nz * x.nr;
  }
  L.buf_elems = e;
  L.fld_elems = fe;
  L.bufA = o; o = align_up(o + es * (size_t)e, 256);
  L.bufB = o; o = align_up(o + es * (size_t)e, 256);
  L.spd = o; o = align_up(o + sizeof(double) * (size_t)align_up(fe, 64), 256);
  // original scheme: two lagged velocity buffers (u_z and u_r of every node)
  L.lag_stride = (d[0].fields & LBAXI_ORIGINAL) ? (long long)align_up(fe, 64) : 0;
  L.lagA = o; o = align_up(o + es * 2 * (size_t)L.lag_stride, 256);
  L.lagB = o; o = align_up(o + es * 2 * (size_t)L.lag_stride, 256);
  L.total = o;
  return L;
}

// Paper-convention relaxation parameters of a descriptor.
void taus(const lbaxi_desc& d, double& tau, double& tau_g, double& tau_h) {
  tau = d.tau - 0.5;
  tau_g = d.tau_g > 0 ? d.tau_g - 0.5 : 2.0 * tau / 3.0;  // tau_g = 2 tau / 3 (Sec. III C)
  tau_h = d.tau_h > 0 ? d.tau_h - 0.5 : tau;
}

lbaxi_status validate(const lbaxi_desc& d, int k) {
  char b[256];
  auto bad = [&](lbaxi_status s, const char* what) {
    snprintf(b, sizeof b, "descriptor %d: %s", k, what);
    return fail(s, b);
  };
  if (d.nz < 2 || d.nr < 2) return bad(LBAXI_EINVAL, "nz and nr must be >= 2");
  // bounds that keep the size arithmetic below in range (any lattice near
  // them is refused by the 4 GiB bound anyway)
  if (d.nz > (1 << 24) || d.nr > (1 << 24)) return bad(LBAXI_EINVAL, "nz and nr must be <= 2^24");
  if (d.prec != LBAXI_FP64 && d.prec != LBAXI_FP32 && d.prec != LBAXI_FP32_FAST)
    return bad(LBAXI_EINVAL, "bad prec");
  if (d.fields & ~255u) return bad(LBAXI_EINVAL, "unknown field bits");
  // element indices inside a lattice are 32-bit (byte offsets stay inside a
  // population's plane, or, in row blocks, below 4 GiB by construction)
  if (lattice_elems(d) >= (1LL << 31))
    return bad(LBAXI_EINVAL, "lattice too large: 2^31 population elements or more");
  if ((d.fields & LBAXI_ZOU_HE) &&
      (!(d.fields & LBAXI_WET_WALLS) || d.west.kind != LBAXI_SIDE_PERIODIC ||
       (d.south.kind == LBAXI_SIDE_WALL && d.south.u_r != 0.0) || d.north.u_r != 0.0))
    return bad(LBAXI_EINVAL,
               "Zou-He walls need wet-node walls, periodic z-ends and no normal wall velocity");
  if ((d.fields & LBAXI_ORIGINAL) &&
      (d.fields & (LBAXI_SWIRL | LBAXI_THERMAL | LBAXI_WET_WALLS | LBAXI_MRT)))
    return bad(LBAXI_EINVAL, "the original scheme models f only, with halfway walls");
  if ((d.fields & LBAXI_WET_WALLS) && (d.nz < 3 || d.nr < 3))
    return bad(LBAXI_EINVAL, "wet-node walls need nz and nr >= 3");
  if (!(d.rho0 > 0)) return bad(LBAXI_EINVAL, "rho0 must be positive");
  if (!(d.r0 >= 0)) return bad(LBAXI_EINVAL, "r0 must be >= 0");
  const lbaxi_side* sd[4] = {&d.south, &d.north, &d.west, &d.east};
  for (int s = 0; s < 4; ++s) {
    const int kd = sd[s]->kind;
    if (kd < 0 || kd > 3) return bad(LBAXI_EINVAL, "bad side kind");
    if (kd == LBAXI_SIDE_AXIS && s != 0) return bad(LBAXI_EINVAL, "axis only as south side");
    if (kd == LBAXI_SIDE_PERIODIC && s < 2) return bad(LBAXI_EINVAL, "periodic only on z-ends");
    if (kd == LBAXI_SIDE_FREESLIP && s < 2) return bad(LBAXI_EINVAL, "free slip only on z-ends");
    if (s >= 2 && sd[s]->r_split >= 0) {
      const int k2 = sd[s]->kind2;
      if (kd == LBAXI_SIDE_PERIODIC || (k2 != LBAXI_SIDE_WALL && k2 != LBAXI_SIDE_FREESLIP))
        return bad(LBAXI_EINVAL, "bad second segment");
    }
  }
  if ((d.west.kind == LBAXI_SIDE_PERIODIC) != (d.east.kind == LBAXI_SIDE_PERIODIC))
    return bad(LBAXI_EINVAL, "periodic must be set on both z-ends");
  if (d.south.kind == LBAXI_SIDE_AXIS && d.r0 != 0.0)
    return bad(LBAXI_EINVAL, "an axis south side needs r0 = 0");
  if (d.south.kind != LBAXI_SIDE_AXIS && !(d.fields & LBAXI_CARTESIAN) && !(d.r0 >= 1.0))
    return bad(LBAXI_EINVAL, "an annulus needs r0 >= 1");
  double tau, tg, th;
  taus(d, tau, tg, th);
  const bool mrt = (d.fields & LBAXI_MRT) != 0;
  if (mrt) {
    const double sr[3] = {d.s_e, d.s_eps, d.s_q};
    for (int q = 0; q < 3; ++q)
      if (!(sr[q] == 0.0 || (sr[q] > 0.0 && sr[q] < 2.0)))
        return bad(LBAXI_ERANGE, "an MRT rate leaves (0, 2)");
  }
  const double tt[3] = {tau, tg, th};
  const bool used[3] = {true, (d.fields & LBAXI_SWIRL) != 0, (d.fields & LBAXI_THERMAL) != 0};
  for (int q = 0; q < 3; ++q) {
    if (!used[q]) continue;
    if (!(tt[q] > 0)) return bad(LBAXI_ERANGE, "relaxation time must exceed 1/2");
    // the MRT rates and the original scheme's rate of f do not depend on r
    if (q == 0 && (mrt || (d.fields & LBAXI_ORIGINAL))) continue;
    for (int j = 0; j < d.nr; ++j) {
      const double r = d.r0 + j;
      const double ir = ((d.fields & LBAXI_CARTESIAN) || r <= 0) ? 0.0 : 1.0 / r;
      for (int e = -1; e <= 1; ++e) {
        const double w = (1.0 + tt[q] * e * ir) / (tt[q] + 0.5);
        if (!(w > 0.0 && w < 2.0))
          return bad(LBAXI_ERANGE, "a relaxation rate leaves (0, 2) on some row");
      }
    }
  }
  return LBAXI_OK;
}

InstP make_inst(const lbaxi_desc& d, long long off, long long off_fld) {
  InstP P;
  memset(&P, 0, sizeof P);
  P.nz = d.nz;
  P.nr = d.nr;
  const PopLayout PL = pop_layout(d);
  P.pitch = (int)PL.pitch;  // row stride
  P.c0 = row_lead(d);
  P.plane = (int)PL.plane;  // population (plane) stride
  P.sw = (int)PL.sw;        // population 0's ghost-column strips
  P.se = (int)PL.se;
  P.cart = (d.fields & LBAXI_CARTESIAN) ? 1 : 0;
  P.wet = (d.fields & LBAXI_WET_WALLS) ? 1 : 0;
  P.zou = (d.fields & LBAXI_ZOU_HE) ? 1 : 0;
  P.r0 = d.r0;
  taus(d, P.tau, P.tau_g, P.tau_h);
  P.rho0 = d.rho0;
  P.mu0 = d.rho0 * P.tau / 3.0;  // mu = tau rho cs^2 (Eq. 36), rho -> rho0
  P.nu_g = P.tau_g / 2.0;        // nu = tau_g c^2 / 2 (Eq. 54)
  P.om0 = 1.0 / (P.tau + 0.5);
  P.omg0 = 1.0 / (P.tau_g + 0.5);
  P.omh0 = 1.0 / (P.tau_h + 0.5);
  // MRT rates: s_e = s_eps = s_v and (1/s_v - 1/2)(1/s_q - 1/2) = 3/16 unless given
  P.s_e = d.s_e > 0 ? d.s_e : P.om0;
  P.s_eps = d.s_eps > 0 ? d.s_eps : P.om0;
  P.s_q = d.s_q > 0 ? d.s_q : 1.0 / (0.5 + 3.0 / (16.0 * P.tau));
  P.a0 = d.a0;
  P.period = d.period;
  P.phase = d.phase;
  P.gbeta = d.gbeta;
  P.T_ref = d.T_ref;
  P.off = off;
  P.off_fld = off_fld;
  const lbaxi_side* sd[4] = {&d.south, &d.north, &d.west, &d.east};
  for (int s = 0; s < 4; ++s) {
    SideP& S = P.side[s];
    S.kind = sd[s]->kind;
    S.thermal = sd[s]->thermal;
    S.kind2 = sd[s]->kind2;
    S.thermal2 = sd[s]->thermal2;
    S.uz = sd[s]->u_z;
    S.ur = sd[s]->u_r;
    S.omega = sd[s]->omega;
    S.T = sd[s]->T;
    S.r_split = (s >= 2) ? sd[s]->r_split : -1.0;
    S.omega2 = sd[s]->omega2;
    S.T2 = sd[s]->T2;
  }
  return P;
}

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

enum { LIST_ALL = 0, LIST_RUN = 1, LIST_HALO = 2 };

}  // namespace

struct lbaxi_s {
  int n = 0, prec = 0;
  unsigned fields = 0;
  bool any_wet = false;  // some lattice has wet-node walls (k_wall runs)
  std::vector<lbaxi_desc> desc;
  std::vector<InstP> ip;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  Layout L;
  InstP* d_ip = nullptr;
  InstDyn* d_dyn = nullptr;
  Tile* d_tiles[3] = {nullptr, nullptr, nullptr};
  int* d_counts = nullptr;  // [LIST_ALL, LIST_RUN, LIST_HALO]
  unsigned long long* d_res = nullptr;
  long long* d_t = nullptr;
  void* bufA = nullptr;
  void* bufB = nullptr;
  void* spd = nullptr;
  void* lagA = nullptr;  // original scheme: lagged velocity, by buffer parity
  void* lagB = nullptr;
  // state of the running lattices (all share parity and time)
  int cur = 0;
  bool pre = true;
  long long t = 0;
  // per lattice
  std::vector<int> status;
  std::vector<InstDyn> dyn;
  std::vector<char> inst_spd;
  bool dyn_dirty = true;
  // launch shape
  int tz = 64, tr = 4, grid = 0, xcd = 0, nt = 1;
  int K = 64;
  int fuse = 1;  // wall part in the step's launch (k_step_wall) where the handle is small
  std::vector<Tile> lists[3];
  int count[3] = {0, 0, 0};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // kernel timing: event pairs around step-kernel launches
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
};

namespace {

void drop_graphs(lbaxi_t* h) {
  for (int q = 0; q < 2; ++q)
    if (h->gexec[q]) {
      (void)hipGraphExecDestroy(h->gexec[q]);
      h->gexec[q] = nullptr;
    }
}

// Rebuild the three work lists for the current shape and statuses, upload
// them (synchronously: the host vectors are reused) and drop stale graphs.
lbaxi_status build_tiles(lbaxi_t* h) {
  for (auto& v : h->lists) v.clear();
  for (int k = 0; k < h->n; ++k) {
    const lbaxi_desc& d = h->desc[k];
    const bool run = h->status[k] == LBAXI_RUNNING;
    for (int j0 = 0; j0 < d.nr; j0 += h->tr)
      for (int i0 = 0; i0 < d.nz; i0 += h->tz) {
        const Tile T = {k, i0, j0, 0};
        h->lists[LIST_ALL].push_back(T);
        if (run) h->lists[LIST_RUN].push_back(T);
      }
    if (run)
      for (int p0 = 0; p0 < perimeter(d); p0 += 256) h->lists[LIST_HALO].push_back(Tile{k, p0, 0, 0});
  }
  int cnt[4] = {0, 0, 0, 0};
  for (int q = 0; q < 3; ++q) {
    h->count[q] = cnt[q] = (int)h->lists[q].size();
    if (cnt[q])
      HIPCHK(hipMemcpyAsync(h->d_tiles[q], h->lists[q].data(), sizeof(Tile) * cnt[q],
                            hipMemcpyHostToDevice, h->stream));
  }
  HIPCHK(hipMemcpyAsync(h->d_counts, cnt, sizeof cnt, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  drop_graphs(h);
  return LBAXI_OK;
}

lbaxi_status upload_dyn(lbaxi_t* h) {
  if (!h->dyn_dirty) return LBAXI_OK;
  for (int k = 0; k < h->n; ++k)
    if (h->status[k] == LBAXI_RUNNING) {
      h->dyn[k].cur = h->cur;
      h->dyn[k].pre = h->pre ? 1 : 0;
      h->dyn[k].t = h->t;
    }
  HIPCHK(hipMemcpyAsync(h->d_dyn, h->dyn.data(), sizeof(InstDyn) * h->n, hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->dyn_dirty = false;
  return LBAXI_OK;
}

template <typename S, typename R, int F>
void* step_fn() { return reinterpret_cast<void*>(&k_step<S, R, F>); }
template <typename S, typename R, int F>
void* step_fn_wetz() {  // the original scheme has no wet-node walls
  if constexpr ((F & F_ORIG) != 0)
    return step_fn<S, R, F>();
  else
    return reinterpret_cast<void*>(&k_step<S, R, F | F_WETZ>);
}
template <typename S, typename R, int F>
void* step_wall_fn() {  // instances with wet-node walls only (the original scheme has none)
  if constexpr ((F & F_ORIG) != 0)
    return nullptr;
  else
    return reinterpret_cast<void*>(&k_step_wall<S, R, F | F_WETZ>);
}
template <typename S, typename R, int F>
void* halo_fn() { return reinterpret_cast<void*>(&k_halo<S, F & 3>); }  // no collision
template <typename S, typename R, int F>
void* wall_fn() { return reinterpret_cast<void*>(&k_wall<S, R, F>); }
template <typename S, typename R, int F>
void* seed_fn() { return reinterpret_cast<void*>(&k_seed<S, R, F>); }
template <typename S, typename R, int F>
void* macros_fn() { return reinterpret_cast<void*>(&k_macros<S, R, F>); }
template <typename S, typename R, int F>
void* resid_fn() { return reinterpret_cast<void*>(&k_residual<S, R, F>); }

// Kernel instance for (precision, field set): FP64 stores and computes in
// double, FP32 stores float and computes in double, FP32_FAST is float only.
#define PICK_B(name, S, R, fields, M)         \
  (((fields) & 3) == 0   ? name<S, R, 0 | M>()  \
   : ((fields) & 3) == 1 ? name<S, R, 1 | M>()  \
   : ((fields) & 3) == 2 ? name<S, R, 2 | M>()  \
                         : name<S, R, 3 | M>())
#define PICK_F(name, S, R, fields)                                      \
  (((fields) & LBAXI_ORIGINAL) ? name<S, R, F_ORIG>()                   \
   : ((fields) & LBAXI_MRT)    ? PICK_B(name, S, R, fields, F_MRT)      \
                               : PICK_B(name, S, R, fields, 0))
#define PICK(name, prec, fields)                                   \
  ((prec) == LBAXI_FP64   ? PICK_F(name, double, double, fields)   \
   : (prec) == LBAXI_FP32 ? PICK_F(name, float, double, fields)    \
                          : PICK_F(name, float, float, fields))

// One step-kernel launch: its function, grid and arguments.  StepArgs has the
// same layout for float and double storage (pointers only).
struct StepLaunch {
  void* fn;
  int grid, block;
  StepArgs<double> a;
};

StepLaunch step_launch(lbaxi_t* h, int list, int from, long long t0, bool use_tdev, int k,
                       int mode) {
  StepLaunch L;
  const bool wetz = h->any_wet && !(h->fields & LBAXI_ORIGINAL);
  L.fn = wetz ? PICK(step_fn_wetz, h->prec, h->fields) : PICK(step_fn, h->prec, h->fields);
  if (wetz) mode |= MODE_WETZ;
  L.block = h->tz * h->tr;
  L.grid = h->grid > 0 ? std::min(h->grid, std::max(1, h->count[list]))
                       : std::max(1, h->count[list]);
  if (h->xcd && L.grid >= 8) L.grid &= ~7;
  StepArgs<double>& a = L.a;
  a.ip = h->d_ip;
  a.tiles = h->d_tiles[list];
  a.ntiles = h->d_counts + list;
  a.src = (const double*)(from ? h->bufB : h->bufA);
  a.dst = (double*)(from ? h->bufA : h->bufB);
  a.spd = (double*)h->spd;
  a.tdev = use_tdev ? h->d_t : nullptr;
  a.t0 = t0;
  a.k = k;
  a.mode = mode;
  a.tzlog = ilog2(h->tz);
  a.tr = h->tr;
  a.xcd = h->xcd;
  a.nt_store = h->nt;
  a.lag_src = (const double*)(from ? h->lagB : h->lagA);
  a.lag_dst = (double*)(from ? h->lagA : h->lagB);
  a.lag_stride = h->L.lag_stride;
  return L;
}

// Wet-wall launch of the same step: the step's arguments over the
// perimeter tiles of the running lattices.
StepLaunch wall_launch(lbaxi_t* h, const StepLaunch& S) {
  StepLaunch W = S;
  W.fn = PICK(wall_fn, h->prec, h->fields);
  W.block = 256;
  W.grid = std::max(1, h->count[LIST_HALO]);
  W.a.tiles = h->d_tiles[LIST_HALO];
  W.a.ntiles = h->d_counts + LIST_HALO;
  return W;
}

// Halo launch filling the ghost slots of buffer `buf` (0 = A, 1 = B).
struct HaloLaunch {
  void* fn;
  int grid;
  const InstP* ip;
  const Tile* tiles;
  const int* ntiles;
  void* buf;
};

HaloLaunch halo_launch(lbaxi_t* h, int buf) {
  HaloLaunch H;
  H.fn = PICK(halo_fn, h->prec, h->fields);
  H.grid = std::max(1, h->count[LIST_HALO]);
  H.ip = h->d_ip;
  H.tiles = h->d_tiles[LIST_HALO];
  H.ntiles = h->d_counts + LIST_HALO;
  H.buf = buf ? h->bufB : h->bufA;
  return H;
}

// Handles with wet-node walls and at most this many perimeter tiles run the
// wall part of each step in the step's launch (k_step_wall).
constexpr int FUSE_MAX_HALO_TILES = 16;

bool fuse_walls(const lbaxi_t* h) {
  return h->fuse && h->any_wet && !(h->fields & LBAXI_ORIGINAL) &&
         h->count[LIST_HALO] <= FUSE_MAX_HALO_TILES;
}

// Step and wall parts as one launch: one workgroup per tile of the step's
// list (whatever the grid option), then one per perimeter tile.
struct StepWallLaunch {
  void* fn;
  int grid, block;
  StepArgs<double> a;
  WallPart b;
};

StepWallLaunch step_wall_launch(lbaxi_t* h, const StepLaunch& L, int list) {
  StepWallLaunch O;
  O.fn = PICK(step_wall_fn, h->prec, h->fields);
  O.block = L.block;
  O.a = L.a;
  O.b.htiles = h->d_tiles[LIST_HALO];
  O.b.nh = h->d_counts + LIST_HALO;
  O.b.ns = std::max(1, h->count[list]);
  O.grid = O.b.ns + std::max(1, h->count[LIST_HALO]);
  return O;
}

// One time step of every running lattice by direct launches: the step kernel
// (the first step after seeding reads each node's own slots, over every
// tile), then the halo fill of the buffer just written.
lbaxi_status launch_step(lbaxi_t* h, int mode) {
  StepLaunch L = h->pre ? step_launch(h, LIST_ALL, h->cur, h->t, false, 0, mode | MODE_PRE)
                        : step_launch(h, LIST_RUN, h->cur, h->t, false, 0, mode);
  void* args[] = {&L.a};
  if (h->prof) {
    while (h->ev.size() < h->ev_used + 2) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->ev.push_back(e);
    }
    HIPCHK(hipEventRecord(h->ev[h->ev_used], h->stream));
  }
  const bool fused = !h->pre && fuse_walls(h);
  if (fused) {
    StepWallLaunch O = step_wall_launch(h, L, LIST_RUN);
    void* oargs[] = {&O.a, &O.b};
    HIPCHK(hipLaunchKernel(O.fn, dim3(O.grid), dim3(O.block), oargs, 0, h->stream));
  } else {
    HIPCHK(hipLaunchKernel(L.fn, dim3(L.grid), dim3(L.block), args, 0, h->stream));
  }
  if (h->prof) {
    HIPCHK(hipEventRecord(h->ev[h->ev_used + 1], h->stream));
    h->ev_used += 2;
  }
  if (h->any_wet && !h->pre && !fused) {
    StepLaunch Wl = wall_launch(h, L);
    void* wargs[] = {&Wl.a};
    HIPCHK(hipLaunchKernel(Wl.fn, dim3(Wl.grid), dim3(Wl.block), wargs, 0, h->stream));
  }
  HaloLaunch H = halo_launch(h, h->cur ^ 1);
  void* hargs[] = {&H.ip, &H.tiles, &H.ntiles, &H.buf};
  HIPCHK(hipLaunchKernel(H.fn, dim3(H.grid), dim3(256), hargs, 0, h->stream));
  h->cur ^= 1;
  h->t += 1;
  h->pre = false;
  return LBAXI_OK;
}

// Graph of K steps starting from buffer `from`: step kernel, halo fill, step
// kernel, ...; a last node advances the device time base by K.
lbaxi_status make_graph(lbaxi_t* h, int from) {
  hipGraph_t g;
  HIPCHK(hipGraphCreate(&g, 0));
  std::vector<hipGraphNode_t> prev;
  lbaxi_status st = LBAXI_OK;
  auto add = [&](void* fn, int grid, int block, void** args) {
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = fn;
    p.gridDim = dim3(grid);
    p.blockDim = dim3(block);
    p.kernelParams = args;
    hipGraphNode_t node;
    hipError_t e =
        hipGraphAddKernelNode(&node, g, prev.empty() ? nullptr : prev.data(), prev.size(), &p);
    if (e != hipSuccess) {
      st = fail(LBAXI_EDEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
      return;
    }
    prev.assign(1, node);
  };
  for (int k = 0; k < h->K && st == LBAXI_OK; ++k) {
    const int src = from ^ (k & 1);
    StepLaunch L = step_launch(h, LIST_RUN, src, 0, true, k, 0);
    if (fuse_walls(h)) {
      StepWallLaunch O = step_wall_launch(h, L, LIST_RUN);
      void* oargs[] = {&O.a, &O.b};
      add(O.fn, O.grid, O.block, oargs);
    } else {
      void* args[] = {&L.a};
      add(L.fn, L.grid, L.block, args);
    }
    if (st != LBAXI_OK) break;
    if (h->any_wet && !fuse_walls(h)) {
      StepLaunch Wl = wall_launch(h, L);
      void* wargs[] = {&Wl.a};
      add(Wl.fn, Wl.grid, Wl.block, wargs);
      if (st != LBAXI_OK) break;
    }
    HaloLaunch H = halo_launch(h, src ^ 1);
    void* hargs[] = {&H.ip, &H.tiles, &H.ntiles, &H.buf};
    add(H.fn, H.grid, 256, hargs);
  }
  if (st == LBAXI_OK) {
    long long* tp = h->d_t;
    long long dv = h->K;
    void* args[] = {&tp, &dv};
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = reinterpret_cast<void*>(&k_add_time);
    p.gridDim = dim3(1);
    p.blockDim = dim3(64);
    p.kernelParams = args;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev.empty() ? nullptr : prev.data(),
                                         prev.size(), &p);
    if (e != hipSuccess)
      st = fail(LBAXI_EDEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
  }
  if (st == LBAXI_OK) {
    hipError_t e = hipGraphInstantiate(&h->gexec[from], g, nullptr, nullptr, 0);
    if (e != hipSuccess)
      st = fail(LBAXI_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  (void)hipGraphDestroy(g);
  return st;
}

lbaxi_status check_handle(const lbaxi_t* h) {
  if (!h) return fail(LBAXI_EINVAL, "NULL handle");
  return LBAXI_OK;
}

lbaxi_status run_steps(lbaxi_t* h, long long n) {
  if (n <= 0) return LBAXI_OK;
  lbaxi_status st;
  if (h->count[LIST_RUN] == 0) return LBAXI_OK;
  long long left = n;
  if (h->pre) {
    if ((st = launch_step(h, left == 1 ? MODE_SPEED : 0)) != LBAXI_OK) return st;
    --left;
  }
  // the last step of the call records |u| for Eq. (57); graphs cover the rest
  if (h->K > 0 && !h->prof && left - 1 >= h->K) {
    const long long reps = (left - 1) / h->K;
    if (!h->gexec[h->cur] && (st = make_graph(h, h->cur)) != LBAXI_OK) return st;
    hipLaunchKernelGGL(k_set_time, dim3(1), dim3(64), 0, h->stream, h->d_t, h->t);
    HIPCHK(hipGetLastError());
    for (long long q = 0; q < reps; ++q) HIPCHK(hipGraphLaunch(h->gexec[h->cur], h->stream));
    h->t += reps * h->K;
    left -= reps * h->K;
  }
  while (left > 0) {
    if ((st = launch_step(h, left == 1 ? MODE_SPEED : 0)) != LBAXI_OK) return st;
    --left;
  }
  h->dyn_dirty = true;
  return LBAXI_OK;
}

// Residual words of every lattice (Eq. 57) reduced into `words` (device
// memory, one 64-bit word per lattice) and copied to out[n] on the host.
// A word holds the bit pattern of a non-negative double (see key), so the
// copy is the residual itself.
lbaxi_status residuals_into(lbaxi_t* h, unsigned long long* words, double* out) {
  lbaxi_status st;
  if ((st = upload_dyn(h)) != LBAXI_OK) return st;
  hipLaunchKernelGGL(k_fill_u64, dim3((h->n + 255) / 256), dim3(256), 0, h->stream, words, h->n,
                     0ULL);
  HIPCHK(hipGetLastError());
  void* fn = PICK(resid_fn, h->prec, h->fields);
  const void* A = h->bufA;
  const void* B = h->bufB;
  const void* S = h->spd;
  unsigned long long* r = words;
  const InstP* ip = h->d_ip;
  const InstDyn* dy = h->d_dyn;
  const Tile* tl = h->d_tiles[LIST_ALL];
  const int* nt = h->d_counts + LIST_ALL;
  int tzlog = ilog2(h->tz);
  Lag lag = {h->lagA, h->lagB, h->L.lag_stride};
  int tile_nodes = h->tz * h->tr;
  void* args[] = {&ip, &dy, &tl, &nt, &A, &B, &S, &r, &tzlog, &tile_nodes, &lag};
  HIPCHK(hipLaunchKernel(fn, dim3(std::max(1, h->count[LIST_ALL])),
                         dim3(std::min(256, tile_nodes)), args, 0, h->stream));
  static_assert(sizeof(double) == sizeof(unsigned long long), "residual words are doubles");
  HIPCHK(hipMemcpyAsync(out, words, sizeof(double) * h->n, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBAXI_OK;
}

lbaxi_status residuals(lbaxi_t* h, std::vector<double>& out) {
  out.resize(h->n);
  return residuals_into(h, h->d_res, out.data());
}

std::mutex g_scratch_mu;
std::map<int, unsigned long long*> g_scratch_ptr;

// Device address of `scratch` on device dev (looked up once per device, with
// that device current).
lbaxi_status scratch_words(int dev, unsigned long long** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return LBAXI_OK;
  }
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != dev) HIPCHK(hipSetDevice(dev));
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) HIPCHK(hipSetDevice(cur));
  if (e != hipSuccess || !ptr)
    return fail(LBAXI_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = static_cast<unsigned long long*>(ptr);
  *out = static_cast<unsigned long long*>(ptr);
  return LBAXI_OK;
}

struct SaveHeader {
  char magic[8];
  int32_t version, n, prec;
  uint32_t fields;
  int64_t t;
  int32_t cur, pre, pad0, pad1;
  uint64_t desc_hash, buf_bytes;
};

uint64_t desc_hash(const std::vector<lbaxi_desc>& d) {
  // FNV-1a over the descriptor bytes (layout-identical handles hash equal)
  uint64_t hsh = 1469598103934665603ULL;
  const unsigned char* p = reinterpret_cast<const unsigned char*>(d.data());
  for (size_t i = 0; i < d.size() * sizeof(lbaxi_desc); ++i) {
    hsh ^= p[i];
    hsh *= 1099511628211ULL;
  }
  return hsh;
}

void freeze(lbaxi_t* h, int k, int status) {
  h->status[k] = status;
  h->dyn[k].cur = h->cur;
  h->dyn[k].pre = h->pre ? 1 : 0;
  h->dyn[k].t = h->t;
  h->dyn_dirty = true;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char* lbaxi_last_error(void) { return g_err.c_str(); }

const char* lbaxi_strerror(lbaxi_status s) {
  switch (s) {
    case LBAXI_OK: return "ok";
    case LBAXI_EINVAL: return "invalid argument";
    case LBAXI_ERANGE: return "relaxation rate out of (0, 2)";
    case LBAXI_ENOMEM: return "workspace too small";
    case LBAXI_EDEVICE: return "HIP error";
    case LBAXI_EDIVERGED: return "diverged (NaN/Inf)";
    case LBAXI_ESTATE: return "invalid state";
    default: return "unknown status";
  }
}

lbaxi_status lbaxi_workspace_bytes(int32_t n, const lbaxi_desc* descs, size_t* bytes) {
  if (n < 1 || !descs || !bytes) return fail(LBAXI_EINVAL, "bad arguments");
  std::vector<lbaxi_desc> d(descs, descs + n);
  for (int k = 0; k < n; ++k) {
    lbaxi_status s = validate(d[k], k);
    if (s != LBAXI_OK) return s;
    const unsigned kset = LBAXI_SWIRL | LBAXI_THERMAL | LBAXI_MRT | LBAXI_ORIGINAL;
    if (d[k].prec != d[0].prec || (d[k].fields & kset) != (d[0].fields & kset))
      return fail(LBAXI_EINVAL,
                  "all lattices of a batch need the same prec, field set and collision model");
  }
  *bytes = layout(d).total;
  return LBAXI_OK;
}

lbaxi_status lbaxi_create(int32_t n, const lbaxi_desc* descs, void* d_workspace, size_t bytes,
                          void* hip_stream, lbaxi_t** out) {
  if (!out) return fail(LBAXI_EINVAL, "NULL out");
  *out = nullptr;
  size_t need = 0;
  lbaxi_status st = lbaxi_workspace_bytes(n, descs, &need);
  if (st != LBAXI_OK) return st;
  if (!d_workspace) return fail(LBAXI_EINVAL, "NULL workspace");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(LBAXI_EINVAL, "workspace not 256-byte aligned");
  if (bytes < need) return fail(LBAXI_ENOMEM, "workspace smaller than lbaxi_workspace_bytes");
  lbaxi_t* h = new (std::nothrow) lbaxi_s();
  if (!h) return fail(LBAXI_ENOMEM, "host allocation failed");
  h->n = n;
  h->desc.assign(descs, descs + n);
  h->prec = descs[0].prec;
  h->fields = descs[0].fields;
  for (int k = 0; k < n; ++k)
    if (descs[k].fields & LBAXI_WET_WALLS) h->any_wet = true;
  // default launch shape: 64 x 4 tiles (one wave along z, 4 rows); 128 x 1
  // where the step kernel's wet-wall instance runs at three waves per SIMD
  // (20 % faster there on the 512 wet melts)
  h->tz = 64;
  h->tr = 4;
  if (h->any_wet && !(h->fields & LBAXI_ORIGINAL)) {
    h->tz = 128;
    h->tr = 1;
  }
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char*>(d_workspace);
  h->L = layout(h->desc);
  h->d_ip = reinterpret_cast<InstP*>(h->ws + h->L.ip);
  h->d_dyn = reinterpret_cast<InstDyn*>(h->ws + h->L.dyn);
  h->d_tiles[LIST_ALL] = reinterpret_cast<Tile*>(h->ws + h->L.tiles_all);
  h->d_tiles[LIST_RUN] = reinterpret_cast<Tile*>(h->ws + h->L.tiles_run);
  h->d_tiles[LIST_HALO] = reinterpret_cast<Tile*>(h->ws + h->L.tiles_halo);
  h->d_counts = reinterpret_cast<int*>(h->ws + h->L.counts);
  h->d_res = reinterpret_cast<unsigned long long*>(h->ws + h->L.res);
  h->d_t = reinterpret_cast<long long*>(h->ws + h->L.tdev);
  h->bufA = h->ws + h->L.bufA;
  h->bufB = h->ws + h->L.bufB;
  h->spd = h->ws + h->L.spd;
  h->lagA = h->ws + h->L.lagA;
  h->lagB = h->ws + h->L.lagB;
  for (int k = 0; k < n; ++k)
    h->ip.push_back(make_inst(h->desc[k], h->L.off[k], h->L.off_fld[k]));
  h->status.assign(n, LBAXI_RUNNING);
  h->dyn.assign(n, InstDyn{0, 1, 0});
  h->inst_spd.assign(n, 0);
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->d_ip, h->ip.data(), sizeof(InstP) * n, hipMemcpyHostToDevice,
                       h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return fail(LBAXI_EDEVICE, std::string("create: ") + hipGetErrorString(e));
  }
  // default launch shape (set above): one workgroup per tile
  st = lbaxi_set_launch(h, h->tz, h->tr, 0, 0, 1);
  if (st == LBAXI_OK) st = lbaxi_seed(h, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (st != LBAXI_OK) {
    lbaxi_destroy(h);
    return st;
  }
  *out = h;
  return LBAXI_OK;
}

void lbaxi_destroy(lbaxi_t* h) {
  if (!h) return;
  drop_graphs(h);
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  delete h;
}

lbaxi_status lbaxi_seed(lbaxi_t* h, const void* d_rho, const void* d_uz, const void* d_ur,
                        const void* d_uth, const void* d_T) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  bool changed = false;
  for (int k = 0; k < h->n; ++k)
    if (h->status[k] != LBAXI_RUNNING) {
      h->status[k] = LBAXI_RUNNING;
      changed = true;
    }
  if (changed && (st = build_tiles(h)) != LBAXI_OK) return st;
  void* fn = PICK(seed_fn, h->prec, h->fields);
  const InstP* ip = h->d_ip;
  const Tile* tl = h->d_tiles[LIST_ALL];
  const int* nt = h->d_counts + LIST_ALL;
  void* buf = h->bufA;
  int tzlog = ilog2(h->tz);
  void* lag = h->lagA;
  long long lag_stride = h->L.lag_stride;
  if (h->fields & LBAXI_ORIGINAL) {
    void* lfn = h->prec == LBAXI_FP64 ? reinterpret_cast<void*>(&k_seed_lag<double>)
                                      : reinterpret_cast<void*>(&k_seed_lag<float>);
    void* largs[] = {&ip, &tl, &nt, &d_uz, &d_ur, &lag, &lag_stride, &tzlog};
    HIPCHK(hipLaunchKernel(lfn, dim3(std::max(1, h->count[LIST_ALL])), dim3(h->tz * h->tr),
                           largs, 0, h->stream));
  }
  void* args[] = {&ip, &tl, &nt, &buf, &d_rho, &d_uz, &d_ur, &d_uth, &d_T, &tzlog, &lag,
                  &lag_stride};
  HIPCHK(hipLaunchKernel(fn, dim3(std::max(1, h->count[LIST_ALL])), dim3(h->tz * h->tr), args,
                         0, h->stream));
  h->cur = 0;
  h->pre = true;
  h->t = 0;
  for (int k = 0; k < h->n; ++k) {
    h->dyn[k] = InstDyn{0, 1, 0};
    h->inst_spd[k] = 0;
  }
  h->dyn_dirty = true;
  return LBAXI_OK;
}

lbaxi_status lbaxi_step(lbaxi_t* h, int64_t n) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (n < 0) return fail(LBAXI_EINVAL, "negative step count");
  st = run_steps(h, n);
  if (st == LBAXI_OK && n > 0)
    for (int k = 0; k < h->n; ++k)
      if (h->status[k] == LBAXI_RUNNING) h->inst_spd[k] = 1;
  return st;
}

lbaxi_status lbaxi_macros(lbaxi_t* h, void* d_rho, void* d_uz, void* d_ur, void* d_uth,
                          void* d_T) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if ((st = upload_dyn(h)) != LBAXI_OK) return st;
  void* fn = PICK(macros_fn, h->prec, h->fields);
  const InstP* ip = h->d_ip;
  const InstDyn* dy = h->d_dyn;
  const Tile* tl = h->d_tiles[LIST_ALL];
  const int* nt = h->d_counts + LIST_ALL;
  const void* A = h->bufA;
  const void* B = h->bufB;
  int tzlog = ilog2(h->tz);
  Lag lag = {h->lagA, h->lagB, h->L.lag_stride};
  int tile_nodes = h->tz * h->tr;
  void* args[] = {&ip,    &dy,   &tl,   &nt,    &A,     &B,          &d_rho,
                  &d_uz,  &d_ur, &d_uth, &d_T, &tzlog, &tile_nodes, &lag};
  HIPCHK(hipLaunchKernel(fn, dim3(std::max(1, h->count[LIST_ALL])),
                         dim3(std::min(256, tile_nodes)), args, 0, h->stream));
  return LBAXI_OK;
}

lbaxi_status lbaxi_residual(lbaxi_t* h, double* host_res) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (!host_res) return fail(LBAXI_EINVAL, "NULL host_res");
  for (int k = 0; k < h->n; ++k)
    if (!h->inst_spd[k]) return fail(LBAXI_ESTATE, "no step since seeding or loading");
  std::vector<double> r;
  if ((st = residuals(h, r)) != LBAXI_OK) return st;
  bool bad = false;
  for (int k = 0; k < h->n; ++k) {
    host_res[k] = r[k];
    if (!std::isfinite(r[k])) bad = true;
  }
  return bad ? fail(LBAXI_EDIVERGED, "NaN or Inf in some lattice") : LBAXI_OK;
}

lbaxi_status lbaxi_residual_static(lbaxi_t* h, double* host_res) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (!host_res) return fail(LBAXI_EINVAL, "NULL host_res");
  if (h->n > STATIC_RESIDUAL_MAX)
    return fail(LBAXI_EINVAL, "lbaxi_residual_static serves handles of at most 8192 lattices");
  for (int k = 0; k < h->n; ++k)
    if (!h->inst_spd[k]) return fail(LBAXI_ESTATE, "no step since seeding or loading");
  unsigned long long* words = nullptr;
  if ((st = scratch_words(h->device, &words)) != LBAXI_OK) return st;
  if ((st = residuals_into(h, words, host_res)) != LBAXI_OK) return st;
  bool bad = false;
  for (int k = 0; k < h->n; ++k)
    if (!std::isfinite(host_res[k])) bad = true;
  return bad ? fail(LBAXI_EDIVERGED, "NaN or Inf in some lattice") : LBAXI_OK;
}

lbaxi_status lbaxi_time(const lbaxi_t* h, int32_t k, int64_t* t) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (k < 0 || k >= h->n || !t) return fail(LBAXI_EINVAL, "bad lattice index");
  *t = h->status[k] == LBAXI_RUNNING ? h->t : h->dyn[k].t;
  return LBAXI_OK;
}

lbaxi_status lbaxi_batch_run(lbaxi_t* h, double tol, int64_t max_steps, int64_t check_every,
                             int32_t* host_status, int64_t* host_steps, double* host_res) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (check_every < 2 || max_steps < 0 || !(tol >= 0) || !host_status || !host_steps)
    return fail(LBAXI_EINVAL, "bad batch_run arguments");
  std::vector<double> last(h->n, -1.0);
  std::vector<long long> t_start(h->n);
  for (int k = 0; k < h->n; ++k) t_start[k] = h->status[k] == LBAXI_RUNNING ? h->t : h->dyn[k].t;
  long long done = 0;
  while (done < max_steps && h->count[LIST_RUN] > 0) {
    const long long n = std::min<long long>(check_every, max_steps - done);
    if ((st = run_steps(h, n)) != LBAXI_OK) return st;
    for (int k = 0; k < h->n; ++k)
      if (h->status[k] == LBAXI_RUNNING) h->inst_spd[k] = 1;
    done += n;
    std::vector<double> r;
    if ((st = residuals(h, r)) != LBAXI_OK) return st;
    bool changed = false;
    for (int k = 0; k < h->n; ++k) {
      if (h->status[k] != LBAXI_RUNNING) continue;
      last[k] = r[k];
      if (!std::isfinite(r[k])) {
        freeze(h, k, LBAXI_DIVERGED);
        changed = true;
      } else if (r[k] <= tol) {
        freeze(h, k, LBAXI_CONVERGED);
        changed = true;
      }
    }
    if (changed && (st = build_tiles(h)) != LBAXI_OK) return st;
  }
  bool capped = false;
  for (int k = 0; k < h->n; ++k) {
    if (h->status[k] == LBAXI_RUNNING && done >= max_steps) {
      freeze(h, k, LBAXI_CAPPED);
      capped = true;
    }
    host_status[k] = h->status[k];
    host_steps[k] = (h->status[k] == LBAXI_RUNNING ? h->t : h->dyn[k].t) - t_start[k];
    if (host_res) host_res[k] = last[k];
  }
  if (capped && (st = build_tiles(h)) != LBAXI_OK) return st;
  return LBAXI_OK;
}

lbaxi_status lbaxi_resume(lbaxi_t* h, int32_t* host_resumed) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  int n = 0;
  for (int k = 0; k < h->n; ++k)
    if (h->status[k] == LBAXI_CAPPED && h->dyn[k].t == h->t && h->dyn[k].cur == h->cur &&
        (h->dyn[k].pre != 0) == h->pre) {
      h->status[k] = LBAXI_RUNNING;
      ++n;
    }
  if (host_resumed) *host_resumed = n;
  if (n) {
    h->dyn_dirty = true;
    return build_tiles(h);
  }
  return LBAXI_OK;
}

lbaxi_status lbaxi_set_launch(lbaxi_t* h, int32_t tile_z, int32_t tile_r, int32_t grid_blocks,
                              int32_t xcd_aware, int32_t nt_store) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (tile_z < 64 || (tile_z & (tile_z - 1)) || tile_r < 1 || tile_z * tile_r > 1024 ||
      grid_blocks < 0)
    return fail(LBAXI_EINVAL, "tile_z must be a power of two >= 64, tile_z*tile_r <= 1024");
  if (h->any_wet && !(h->fields & LBAXI_ORIGINAL) && tile_z * tile_r > 512)
    return fail(LBAXI_EINVAL, "handles with wet-node walls take tile_z*tile_r <= 512");
  h->tz = tile_z;
  h->tr = tile_r;
  h->grid = grid_blocks;
  h->xcd = xcd_aware ? 1 : 0;
  h->nt = nt_store ? 1 : 0;
  return build_tiles(h);
}

lbaxi_status lbaxi_get_launch(const lbaxi_t* h, int32_t* cfg5) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (!cfg5) return fail(LBAXI_EINVAL, "NULL cfg5");
  cfg5[0] = h->tz;
  cfg5[1] = h->tr;
  cfg5[2] = h->grid;
  cfg5[3] = h->xcd;
  cfg5[4] = h->nt;
  return LBAXI_OK;
}

lbaxi_status lbaxi_set_fused_walls(lbaxi_t* h, int32_t on) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (on != 0 && on != 1) return fail(LBAXI_EINVAL, "set_fused_walls: on must be 0 or 1");
  h->fuse = on;
  drop_graphs(h);
  return LBAXI_OK;
}

lbaxi_status lbaxi_set_graph_steps(lbaxi_t* h, int32_t k) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (k < 0 || (k & 1)) return fail(LBAXI_EINVAL, "graph length must be even and >= 0");
  h->K = k;
  drop_graphs(h);
  return LBAXI_OK;
}

lbaxi_status lbaxi_autotune(lbaxi_t* h, int32_t steps_per_trial, int32_t* cfg5_out) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (steps_per_trial < 2) return fail(LBAXI_EINVAL, "steps_per_trial must be >= 2");
  static const int shapes[][2] = {{64, 1}, {64, 2}, {64, 4}, {64, 8}, {128, 1},
                                  {128, 2}, {128, 4}, {256, 1}, {256, 2}, {512, 1}};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int dev_cu = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) dev_cu = prop.multiProcessorCount;
  }
  auto trial = [&](int tz, int tr, int grid, int xcd, int nt, float& ms) -> lbaxi_status {
    lbaxi_status s = lbaxi_set_launch(h, tz, tr, grid, xcd, nt);
    if (s != LBAXI_OK) return s;
    if ((s = run_steps(h, 2)) != LBAXI_OK) return s;  // warm-up + graph build
    HIPCHK(hipEventRecord(e0, h->stream));
    if ((s = run_steps(h, steps_per_trial)) != LBAXI_OK) return s;
    HIPCHK(hipEventRecord(e1, h->stream));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return LBAXI_OK;
  };
  float best = 1e30f;
  int b[5] = {h->tz, h->tr, h->grid, h->xcd, h->nt};
  // one workgroup per tile, dealt round-robin over the XCDs (xcd = 0) or in
  // eight contiguous bands, one per XCD (xcd = 1: z-adjacent tiles, which
  // share the cache lines at their common edge, then meet in one L2)
  for (const auto& sh : shapes)
    for (int xcd = 0; xcd < 2 && st == LBAXI_OK; ++xcd) {
      float ms;
      if ((st = trial(sh[0], sh[1], 0, xcd, 1, ms)) != LBAXI_OK) break;
      if (ms < best) {
        best = ms;
        b[0] = sh[0]; b[1] = sh[1]; b[2] = 0; b[3] = xcd; b[4] = 1;
      }
    }
  if (st == LBAXI_OK) {
    const int wg = b[0] * b[1];
    const int per_cu = std::max(1, 2048 / wg);
    const int grids[] = {dev_cu * per_cu, dev_cu * per_cu * 2, dev_cu * per_cu / 2};
    const int base[2] = {b[0], b[1]};
    for (int gi = 0; gi < 3 && st == LBAXI_OK; ++gi)
      for (int xcd = 0; xcd < 2 && st == LBAXI_OK; ++xcd) {
        float ms;
        if ((st = trial(base[0], base[1], grids[gi], xcd, 1, ms)) != LBAXI_OK) break;
        if (ms < best) {
          best = ms;
          b[2] = grids[gi]; b[3] = xcd; b[4] = 1;
        }
      }
    float ms;
    if (st == LBAXI_OK && (st = trial(b[0], b[1], b[2], b[3], 0, ms)) == LBAXI_OK && ms < best) {
      best = ms;
      b[4] = 0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LBAXI_OK) return st;
  h->dyn_dirty = true;
  for (int k = 0; k < h->n; ++k)
    if (h->status[k] == LBAXI_RUNNING) h->inst_spd[k] = 1;
  if ((st = lbaxi_set_launch(h, b[0], b[1], b[2], b[3], b[4])) != LBAXI_OK) return st;
  if (cfg5_out) memcpy(cfg5_out, b, sizeof b);
  return LBAXI_OK;
}

lbaxi_status lbaxi_state_bytes(const lbaxi_t* h, size_t* bytes) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (!bytes) return fail(LBAXI_EINVAL, "NULL bytes");
  *bytes = sizeof(SaveHeader) + sizeof(InstDyn) * h->n + sizeof(int32_t) * h->n +
           sizeof(char) * h->n + elem_size(h->prec) * (size_t)h->L.buf_elems +
           sizeof(double) * (size_t)h->L.fld_elems +
           elem_size(h->prec) * 2 * (size_t)h->L.lag_stride;
  return LBAXI_OK;
}

lbaxi_status lbaxi_save(lbaxi_t* h, void* host_buf, size_t bytes) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  size_t need;
  if ((st = lbaxi_state_bytes(h, &need)) != LBAXI_OK) return st;
  if (!host_buf || bytes < need) return fail(LBAXI_EINVAL, "save buffer too small");
  for (int k = 0; k < h->n; ++k)
    if (h->status[k] == LBAXI_RUNNING) {
      h->dyn[k].cur = h->cur;
      h->dyn[k].pre = h->pre;
      h->dyn[k].t = h->t;
    }
  const size_t es = elem_size(h->prec);
  char* p = static_cast<char*>(host_buf);
  SaveHeader H;
  memset(&H, 0, sizeof H);
  memcpy(H.magic, "LBAXISV3", 8);  // V3: row-blocked population layout
  H.version = 3;
  H.n = h->n;
  H.prec = h->prec;
  H.fields = h->fields;
  H.t = h->t;
  H.cur = h->cur;
  H.pre = h->pre;
  H.desc_hash = desc_hash(h->desc);
  H.buf_bytes = es * (size_t)h->L.buf_elems;
  memcpy(p, &H, sizeof H);
  p += sizeof H;
  memcpy(p, h->dyn.data(), sizeof(InstDyn) * h->n);
  p += sizeof(InstDyn) * h->n;
  memcpy(p, h->status.data(), sizeof(int32_t) * h->n);
  p += sizeof(int32_t) * h->n;
  memcpy(p, h->inst_spd.data(), h->n);
  p += h->n;
  // every lattice's own current buffer, instance by instance
  for (int k = 0; k < h->n; ++k) {
    const char* src =
        static_cast<const char*>(h->dyn[k].cur ? h->bufB : h->bufA) + es * h->L.off[k];
    const size_t nb = es * (size_t)lattice_elems(h->desc[k]);
    HIPCHK(hipMemcpyAsync(p + es * h->L.off[k], src, nb, hipMemcpyDeviceToHost, h->stream));
  }
  p += es * (size_t)h->L.buf_elems;
  HIPCHK(hipMemcpyAsync(p, h->spd, sizeof(double) * (size_t)h->L.fld_elems,
                        hipMemcpyDeviceToHost, h->stream));
  p += sizeof(double) * (size_t)h->L.fld_elems;
  // original scheme: each lattice's lagged velocity (buffer of its parity)
  const long long ls = h->L.lag_stride;
  for (int k = 0; k < h->n && ls > 0; ++k) {
    const char* src = static_cast<const char*>(h->dyn[k].cur ? h->lagB : h->lagA);
    const size_t o = es * (size_t)h->L.off_fld[k];
    const size_t nb = es * (size_t)h->desc[k].nz * h->desc[k].nr;
    HIPCHK(hipMemcpyAsync(p + o, src + o, nb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(p + es * ls + o, src + es * ls + o, nb, hipMemcpyDeviceToHost,
                          h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBAXI_OK;
}

lbaxi_status lbaxi_load(lbaxi_t* h, const void* host_buf, size_t bytes) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  size_t need;
  if ((st = lbaxi_state_bytes(h, &need)) != LBAXI_OK) return st;
  if (!host_buf || bytes < need) return fail(LBAXI_EINVAL, "load buffer too small");
  const char* p = static_cast<const char*>(host_buf);
  SaveHeader H;
  memcpy(&H, p, sizeof H);
  if (memcmp(H.magic, "LBAXISV3", 8) || H.n != h->n || H.prec != h->prec ||
      H.fields != h->fields || H.desc_hash != desc_hash(h->desc))
    return fail(LBAXI_EINVAL, "checkpoint does not match this handle");
  p += sizeof H;
  memcpy(h->dyn.data(), p, sizeof(InstDyn) * h->n);
  p += sizeof(InstDyn) * h->n;
  memcpy(h->status.data(), p, sizeof(int32_t) * h->n);
  p += sizeof(int32_t) * h->n;
  memcpy(h->inst_spd.data(), p, h->n);
  p += h->n;
  const size_t es = elem_size(h->prec);
  for (int k = 0; k < h->n; ++k) {
    char* dst = static_cast<char*>(h->dyn[k].cur ? h->bufB : h->bufA) + es * h->L.off[k];
    const size_t nb = es * (size_t)lattice_elems(h->desc[k]);
    HIPCHK(hipMemcpyAsync(dst, p + es * h->L.off[k], nb, hipMemcpyHostToDevice, h->stream));
  }
  p += es * (size_t)h->L.buf_elems;
  HIPCHK(hipMemcpyAsync(h->spd, p, sizeof(double) * (size_t)h->L.fld_elems,
                        hipMemcpyHostToDevice, h->stream));
  p += sizeof(double) * (size_t)h->L.fld_elems;
  const long long ls = h->L.lag_stride;
  for (int k = 0; k < h->n && ls > 0; ++k) {
    char* dst = static_cast<char*>(h->dyn[k].cur ? h->lagB : h->lagA);
    const size_t o = es * (size_t)h->L.off_fld[k];
    const size_t nb = es * (size_t)h->desc[k].nz * h->desc[k].nr;
    HIPCHK(hipMemcpyAsync(dst + o, p + o, nb, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(dst + es * ls + o, p + es * ls + o, nb, hipMemcpyHostToDevice,
                          h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  h->t = H.t;
  h->cur = H.cur;
  h->pre = H.pre != 0;
  h->dyn_dirty = true;
  return build_tiles(h);
}

lbaxi_status lbaxi_node_count(const lbaxi_t* h, int64_t* nodes, int32_t* n) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (nodes) *nodes = h->L.fld_elems;
  if (n) *n = h->n;
  return LBAXI_OK;
}

size_t lbaxi_abi_desc_size(void) { return sizeof(lbaxi_desc); }

lbaxi_status lbaxi_set_profiling(lbaxi_t* h, int32_t on) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  h->prof = on != 0;
  return LBAXI_OK;
}

lbaxi_status lbaxi_kernel_time(lbaxi_t* h, double* ms, int64_t* launches) {
  lbaxi_status st = check_handle(h);
  if (st != LBAXI_OK) return st;
  if (!ms || !launches) return fail(LBAXI_EINVAL, "NULL output");
  HIPCHK(hipStreamSynchronize(h->stream));
  double total = 0;
  for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
    float e = 0;
    HIPCHK(hipEventElapsedTime(&e, h->ev[k], h->ev[k + 1]));
    total += e;
  }
  *ms = total;
  *launches = (int64_t)(h->ev_used / 2);
  h->ev_used = 0;
  return LBAXI_OK;
}

lbaxi_status lbaxi_stream_copy(const void* d_src, void* d_dst, size_t bytes, int32_t loads_per_lane,
                               void* hip_stream) {
  if (!d_src || !d_dst || bytes % 16 || (reinterpret_cast<uintptr_t>(d_src) % 16) ||
      (reinterpret_cast<uintptr_t>(d_dst) % 16))
    return fail(LBAXI_EINVAL, "copy needs 16-byte aligned pointers and size");
  const int U = loads_per_lane;
  if (U != 1 && U != 2 && U != 4 && U != 8) return fail(LBAXI_EINVAL, "loads_per_lane must be 1, 2, 4 or 8");
  const long long n = (long long)(bytes / 16);
  if (n == 0) return LBAXI_OK;
  const long long grid = (n + 256LL * U - 1) / (256LL * U);
  if (grid > 0x7fffffffLL) return fail(LBAXI_EINVAL, "copy larger than 2^31 workgroups");
  const hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const u32x4* a = static_cast<const u32x4*>(d_src);
  u32x4* b = static_cast<u32x4*>(d_dst);
  switch (U) {
    case 1: hipLaunchKernelGGL(k_copy<1>, dim3((unsigned)grid), dim3(256), 0, st, a, b, n); break;
    case 2: hipLaunchKernelGGL(k_copy<2>, dim3((unsigned)grid), dim3(256), 0, st, a, b, n); break;
    case 4: hipLaunchKernelGGL(k_copy<4>, dim3((unsigned)grid), dim3(256), 0, st, a, b, n); break;
    default: hipLaunchKernelGGL(k_copy<8>, dim3((unsigned)grid), dim3(256), 0, st, a, b, n); break;
  }
  HIPCHK(hipGetLastError());
  return LBAXI_OK;
}

}  // extern "C"
