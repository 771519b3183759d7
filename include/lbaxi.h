/*
 * lbaxi.h -- C ABI of the MI355X (gfx950) improved axisymmetric lattice
 * Boltzmann library (Li, He, Tang, Tao, arXiv:1003.0282).
 *
 * The library advances, on one GPU, one or many independent lattices on the
 * (z, r) meridian plane:
 *   f : D2Q9 populations of the improved BGK scheme, Eq. (13) with the
 *       gradient-free source of Eq. (12), the direction-dependent relaxation
 *       rate omega_f = (1 + tau e_r / r)/(tau + 1/2) and the macros of
 *       Eqs. (16)-(17) (Sec. III A).  With LBAXI_MRT f collides instead with
 *       the MRT model of Sec. III B: moments of Eq. (38), Eq. (41) on f-bar =
 *       f - S/2 (Eq. 40) with the source of Eq. (51), and the momentum rows
 *       modified by Eqs. (49)-(50) to carry the 1/r viscous terms; the
 *       macros stay Eqs. (16)-(17);
 *   g : D2Q4 azimuthal-velocity populations, Eqs. (53)-(54) (Sec. III C),
 *       optional (LBAXI_SWIRL);
 *   h : D2Q4 temperature populations built like Eqs. (53)-(54) with source
 *       -(u_r / r) h_eq and Boussinesq buoyancy on the axial force (the paper
 *       defines no temperature scheme; this one is an assumption), optional
 *       (LBAXI_THERMAL).
 * The axis r = 0 is a node row on which every 1/r term is zero; f and h are
 * specularly reflected there and g takes the non-equilibrium extrapolation of
 * its radial neighbour (Sec. IV A-B).  Walls are halfway bounce-back links
 * (moving-wall term for f, anti-bounce-back for the Dirichlet values of g and
 * h).  Steady convergence is measured by Eq. (57).
 *
 * Conventions
 *   - Node (i, j): i = 0..nz-1 along z, j = 0..nr-1 along r, r_j = r0 + j.
 *     A field is an array [nr][nz] with z fastest.  A batch of instances
 *     packs their fields one after another in instance order.
 *   - tau, tau_g, tau_h are BGK relaxation times tau_s = paper tau + 1/2
 *     (kinematic viscosity nu = (tau_s - 1/2)/3).  tau_g = 0 selects the
 *     paper's tau_g = 2 tau / 3 (paper convention); tau_h = 0 selects tau_h =
 *     tau.
 *   - Device pointers ("d_") are caller-owned device memory; host pointers
 *     ("host_") are caller-owned host memory.  The library never allocates
 *     device memory: all device state lives in the caller's workspace, which
 *     must stay allocated and untouched until lbaxi_destroy.  The library
 *     owns only its host-side handle and the HIP graphs it instantiates.
 *   - All work is enqueued on the caller's HIP stream given at creation;
 *     functions that return host data synchronise that stream.  A handle is
 *     not thread-safe and must be used from one host thread at a time.
 *   - Every function returns LBAXI_OK (0) or a negative status; no C++
 *     exception crosses this boundary.  lbaxi_last_error() gives a message.
 */
#ifndef LBAXI_H
#define LBAXI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbaxi_status;
enum {
  LBAXI_OK = 0,
  LBAXI_EINVAL = -1,    /* invalid argument or descriptor */
  LBAXI_ERANGE = -2,    /* a relaxation rate leaves (0, 2) on some row */
  LBAXI_ENOMEM = -3,    /* workspace too small */
  LBAXI_EDEVICE = -4,   /* a HIP call failed */
  LBAXI_EDIVERGED = -5, /* NaN / Inf seen by the residual */
  LBAXI_ESTATE = -6     /* call not valid in the current state */
};

/* Precision of a handle.  FP64: populations stored and computed in double.
 * FP32: populations stored in float (as deviations from w_a rho0), every
 * node update computed in double -- FP32 rounding inside the update, not in
 * storage, is what limits a float path on slowly converging flows.
 * FP32_FAST: stored and computed in float.  Fields passed to lbaxi_seed and
 * returned by lbaxi_macros are double for FP64 and float otherwise. */
enum { LBAXI_FP64 = 0, LBAXI_FP32 = 1, LBAXI_FP32_FAST = 2 };
/* Field set and wall model bits of lbaxi_desc.fields.  LBAXI_WET_WALLS puts
 * every wall side (radial walls and z-end wall / free-slip segments) through
 * the outermost node row or column and rebuilds those nodes after each step
 * by non-equilibrium extrapolation from their inner neighbour, the paper's
 * wall treatment of its rotating flows (Sec. IV B); without it walls are
 * halfway links half a spacing outside the last node.  The wall node keeps
 * the mass it streamed in (no mass crosses the wall); its velocity, u_theta
 * and T (fixed-temperature walls) take the wall values.  Needs nz, nr >= 3.
 * LBAXI_MRT selects the MRT collision of f (Sec. III B; rates in
 * lbaxi_desc.s_e, s_eps, s_q, with s_v = 1/tau fixed by the viscosity);
 * seeding and wet-node walls then use its source, S = M^-1 S~.
 * LBAXI_ORIGINAL runs instead the original scheme the paper improves on
 * (Sec. II): Eq. (8) with the constant rate 1/(tau + 1/2), the source of
 * Eq. (7) and the macros of Eqs. (9)-(10), whose velocity-gradient terms are
 * central differences of the previous level's velocity (the handle keeps
 * that field: 2 values per node more in the workspace, read and written
 * each step).  f only: not with SWIRL, THERMAL, WET_WALLS or MRT.
 * LBAXI_ZOU_HE (with LBAXI_WET_WALLS) rebuilds f on the radial wall nodes by
 * Zou and He's no-slip rule, the paper's wall treatment of its pipe flows
 * (Sec. IV A, its Ref. 47): the populations from beyond the wall follow from
 * Eqs. (16)-(17) at the wall velocity and non-equilibrium bounce-back along
 * the normal; g and h keep the extrapolation.  Only with periodic z-ends
 * (the paper's pipes: where a Zou-He wall met an extrapolated z-end wall
 * the corner went unstable at small tau) and radial walls without normal
 * velocity (u_r = 0); EINVAL otherwise.  Zou-He walls are not robust at
 * small tau: started from noisy states they diverged at tau <= 0.55. */
enum {
  LBAXI_SWIRL = 1u,
  LBAXI_THERMAL = 2u,
  LBAXI_CARTESIAN = 4u,
  LBAXI_WET_WALLS = 8u,
  LBAXI_MRT = 16u,
  LBAXI_ORIGINAL = 32u,
  LBAXI_ZOU_HE = 64u,
  /* Memory layout of this lattice's populations: each population's rows
   * contiguous (planes) instead of the default row blocks (the rows of all
   * populations of one lattice row side by side, which the step kernel
   * streams faster).  Same results bit for bit.  A lattice whose row
   * blocks would take 4 GiB or more is stored as planes anyway. */
  LBAXI_PLANES = 128u
};
enum {
  LBAXI_SIDE_AXIS = 0,     /* south side only, r0 = 0: specular axis */
  LBAXI_SIDE_WALL = 1,     /* halfway bounce-back wall */
  LBAXI_SIDE_PERIODIC = 2, /* west and east together */
  LBAXI_SIDE_FREESLIP = 3  /* z-ends only: specular wall (f), zero flux (g, h) */
};
/* Per-instance run status reported by lbaxi_batch_run. */
enum { LBAXI_RUNNING = 0, LBAXI_CONVERGED = 1, LBAXI_DIVERGED = 2, LBAXI_CAPPED = 3 };

/* One side of the rectangle.  south: r = r0 - 1/2 (or the axis row when
 * r0 = 0), north: r = r0 + nr - 1/2, west: z = -1/2, east: z = nz - 1/2.
 * A z-end (west/east) may carry a second segment for nodes with r_j >
 * r_split (e.g. a crystal disk and a free surface beside it); r_split < 0
 * disables it.  Radial sides ignore the second segment. */
typedef struct {
  int32_t kind;     /* LBAXI_SIDE_* */
  int32_t thermal;  /* 1: fixed temperature T, 0: adiabatic */
  double u_z, u_r;  /* wall velocity in the meridian plane (f) */
  double omega;     /* wall angular speed; u_theta at the wall = omega * r */
  double T;         /* wall temperature when thermal = 1 */
  double r_split;   /* see above */
  int32_t kind2;    /* second segment: LBAXI_SIDE_WALL or _FREESLIP */
  int32_t thermal2;
  double omega2;
  double T2;
} lbaxi_side;

typedef struct {
  int32_t nz, nr;   /* nodes along z and r, each >= 2 */
  double r0;        /* radius of node row 0; 0 with an axis south side */
  int32_t prec;     /* LBAXI_FP64 / _FP32 / _FP32_FAST (same for a whole batch) */
  uint32_t fields;  /* LBAXI_SWIRL | _THERMAL | _CARTESIAN | _WET_WALLS | _MRT | _ORIGINAL | _PLANES
                       | _ZOU_HE */
  double tau;       /* tau_s of f */
  double tau_g;     /* tau_s of g, 0 -> paper default */
  double tau_h;     /* tau_s of h, 0 -> tau */
  double rho0;      /* reference density (incompressible limit, Sec. III A) */
  double a0, period, phase; /* axial force density a0 cos(2 pi t/period + phase);
                               period <= 0: constant a0 */
  double gbeta, T_ref;      /* buoyancy rho0 * gbeta * (T - T_ref) along +z */
  lbaxi_side south, north, west, east;
  /* MRT relaxation rates (used with LBAXI_MRT only) of the moments e,
   * epsilon and q of Eq. (38); 0 selects the default: s_e = s_eps = s_v
   * (the paper requires s_e = s_v, Sec. III B) and s_q from
   * (1/s_v - 1/2)(1/s_q - 1/2) = 3/16.  The conserved moments need no rate:
   * with f-bar = f - S/2 they leave the collision as m-bar + S~ for any. */
  double s_e, s_eps, s_q;
} lbaxi_desc;

typedef struct lbaxi_s lbaxi_t; /* opaque handle */

/* Text of the most recent error on the calling thread (never NULL). */
const char* lbaxi_last_error(void);
const char* lbaxi_strerror(lbaxi_status s);

/* Device workspace needed by a batch of n descriptors (n = 1: one lattice).
 * Sec. III A: state is two population buffers (ping-pong) plus one speed
 * field per lattice for Eq. (57).  A buffer holds each lattice's populations
 * in row blocks (the padded rows of all Q populations of one lattice row,
 * one after the other, for rows -1..nr, then two blocks of z-end ghost
 * columns), or, with LBAXI_PLANES and for lattices whose row blocks would
 * take 4 GiB or more, in planes (each population's rows contiguous); one
 * lattice may hold fewer than 2^31 population elements, EINVAL beyond. */
lbaxi_status lbaxi_workspace_bytes(int32_t n, const lbaxi_desc* descs, size_t* bytes);

/* Create a handle over n lattices (all the same prec, the same SWIRL and
 * THERMAL bits and the same scheme (BGK, MRT or ORIGINAL); CARTESIAN and
 * WET_WALLS may differ between lattices), carving
 * d_workspace (>= lbaxi_workspace_bytes, 256-byte aligned) and enqueuing on
 * hip_stream (a hipStream_t; NULL = the null stream).  Validates every
 * descriptor: EINVAL for bad sizes (2^31 population elements or more in
 * one lattice included) or side combinations (axis only as south
 * with r0 = 0, periodic only on both z-ends together, free slip only on
 * z-ends), ERANGE when some relaxation rate (1 + tau e_r / r)/(tau + 1/2) of
 * f (BGK), g or h, or an MRT rate, leaves (0, 2).  The lattices start at rest (lbaxi_seed with NULL
 * fields). */
lbaxi_status lbaxi_create(int32_t n, const lbaxi_desc* descs, void* d_workspace,
                          size_t bytes, void* hip_stream, lbaxi_t** out);
void lbaxi_destroy(lbaxi_t* h);

/* Equilibrium seeding of every lattice (Eq. 6 and Eq. 54; the paper starts
 * from rest): f^ = f_eq(rho, u) - S(rho, u)/2 with S of Eq. (12) (with
 * LBAXI_MRT the velocity-space MRT source M^-1 S~; with LBAXI_ORIGINAL the
 * G of Eq. (7), its gradient terms taken from the given velocity field),
 * g = g_eq, h = h_eq, so the macros return the given fields.  Each d_ pointer is a
 * packed field set of the handle's precision (double for FP64, float for
 * FP32), or NULL for rho0 / zero velocity / T_ref.  u_r and u_theta are
 * forced to 0 on an axis row.  Resets the time to 0 and every status to
 * RUNNING.  The fields are read by a kernel on the handle's stream: they must
 * stay valid until that stream has passed this call. */
lbaxi_status lbaxi_seed(lbaxi_t* h, const void* d_rho, const void* d_uz, const void* d_ur,
                        const void* d_uth, const void* d_T);

/* Advance every RUNNING lattice by n >= 0 time steps (asynchronous).  One
 * step = pull streaming with the boundary rules + macros (Eqs. 16-17) +
 * collision (Eqs. 12-13, or the MRT or original model the handle selects,
 * and 53-54).  Long runs replay a captured HIP graph. */
lbaxi_status lbaxi_step(lbaxi_t* h, int64_t n);

/* Macroscopic fields at the current time level (Eqs. 16-17, or Eqs. 9-10 with
 * LBAXI_ORIGINAL; u_theta = sum g / rho0, T = sum h), packed over all
 * lattices; any pointer may be
 * NULL.  Element type = the handle's precision.  Asynchronous. */
lbaxi_status lbaxi_macros(lbaxi_t* h, void* d_rho, void* d_uz, void* d_ur, void* d_uth,
                          void* d_T);

/* Eq. (57): max over nodes of | |u|(t) - |u|(t-1) |, with t the current
 * level, for every lattice (host_res[n]).  Synchronises the stream.  Returns
 * LBAXI_EDIVERGED (and NaN entries) when any lattice holds NaN or Inf, and
 * LBAXI_ESTATE when no step has been taken since seeding or loading. */
lbaxi_status lbaxi_residual(lbaxi_t* h, double* host_res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid it): lbaxi_residual with its
 * per-lattice reduction words in a fixed array of the library's device memory
 * (64 KiB per GPU, held until the process ends) instead of the handle's
 * workspace.  Same results and statuses as lbaxi_residual; EINVAL for a handle
 * of more than 8192 lattices.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other host threads, other streams) race. */
lbaxi_status lbaxi_residual_static(lbaxi_t* h, double* host_res);

/* Current time level of lattice k. */
lbaxi_status lbaxi_time(const lbaxi_t* h, int32_t k, int64_t* t);

/* Run every lattice until its residual (Eq. 57) is <= tol (CONVERGED), it
 * turns NaN/Inf (DIVERGED) or it has taken max_steps steps (CAPPED),
 * checking every check_every steps; finished lattices stop stepping while
 * the others go on in the same launches.  host_status[n] and host_steps[n]
 * receive the outcome; host_res[n] (may be NULL) the last residual. */
lbaxi_status lbaxi_batch_run(lbaxi_t* h, double tol, int64_t max_steps, int64_t check_every,
                             int32_t* host_status, int64_t* host_steps, double* host_res);

/* Let CAPPED lattices that stopped together with the last running ones
 * (same time level) run again in the next lbaxi_step / lbaxi_batch_run, so
 * that a long run can be split into calls; *host_resumed (may be NULL)
 * receives their number. */
lbaxi_status lbaxi_resume(lbaxi_t* h, int32_t* host_resumed);

/* Launch shape of the fused step kernel: tile_z x tile_r nodes per
 * workgroup (tile_z a power of two >= 64, tile_z * tile_r <= 1024, or <= 512
 * on a handle with wet-node walls, whose step kernel also rebuilds the
 * z-end wall nodes; EINVAL otherwise; default 64 x 4, or 128 x 1 on a
 * handle with wet-node walls), grid_blocks
 * persistent workgroups (0 = one workgroup per tile), xcd_aware = 1 gives
 * each of the 8 XCDs a contiguous band of tiles, nt_store = 1 uses
 * non-temporal stores for the populations. */
lbaxi_status lbaxi_set_launch(lbaxi_t* h, int32_t tile_z, int32_t tile_r, int32_t grid_blocks,
                              int32_t xcd_aware, int32_t nt_store);
lbaxi_status lbaxi_get_launch(const lbaxi_t* h, int32_t* cfg5);

/* Length K (even, >= 0) of the HIP graph replayed for long runs; 0 disables
 * graphs (every step is a direct launch).  Default 64. */
lbaxi_status lbaxi_set_graph_steps(lbaxi_t* h, int32_t k);

/* Wet-node walls of small handles (on = 1, the default): for a handle with
 * LBAXI_WET_WALLS lattices whose running lattices have at most 16 x 256
 * perimeter nodes in all, the wall-node rebuild (Sec. IV B's
 * non-equilibrium extrapolation) runs in the step kernel's launch, as
 * further workgroups, instead of a launch of its own: one launch fewer per
 * step.  on = 0 keeps the separate launch.  Bitwise the same results
 * either way; no effect on other handles.  EINVAL for other values. */
lbaxi_status lbaxi_set_fused_walls(lbaxi_t* h, int32_t on);

/* Autotuner: times each candidate launch shape over steps_per_trial real
 * time steps (the steps count: the state advances) and keeps the fastest;
 * cfg5_out (may be NULL) receives it.  Synchronises the stream. */
lbaxi_status lbaxi_autotune(lbaxi_t* h, int32_t steps_per_trial, int32_t* cfg5_out);

/* Checkpoint: raw populations of the current level plus time and status (and,
 * with LBAXI_ORIGINAL, the lagged velocity field the next step needs).
 * lbaxi_state_bytes gives the size; lbaxi_save copies to host memory
 * (synchronising), lbaxi_load restores a state saved by a handle created
 * from identical descriptors (EINVAL otherwise). */
lbaxi_status lbaxi_state_bytes(const lbaxi_t* h, size_t* bytes);
lbaxi_status lbaxi_save(lbaxi_t* h, void* host_buf, size_t bytes);
lbaxi_status lbaxi_load(lbaxi_t* h, const void* host_buf, size_t bytes);

/* Kernel timing for roofline fractions.  With profiling on, steps are
 * launched one by one (no graph replay) and a pair of HIP events on the
 * handle's stream brackets every launch of the fused step kernel.
 * lbaxi_kernel_time synchronises the stream and returns the summed duration
 * (ms) and the number of step-kernel launches since the previous call. */
lbaxi_status lbaxi_set_profiling(lbaxi_t* h, int32_t on);
lbaxi_status lbaxi_kernel_time(lbaxi_t* h, double* ms, int64_t* launches);

/* sizeof(lbaxi_desc) as compiled into the library, for binding checks. */
size_t lbaxi_abi_desc_size(void);

/* Sum of nr * nz over the handle's lattices and the number of lattices. */
lbaxi_status lbaxi_node_count(const lbaxi_t* h, int64_t* nodes, int32_t* n);

/* Plain device-to-device streaming copy of `bytes` (a multiple of 16, both
 * pointers 16-byte aligned) on hip_stream: the bandwidth reference used to
 * calibrate HBM counters and to measure the streaming ceiling the step kernel
 * is compared with.  loads_per_lane (1, 2, 4 or 8) 16-byte loads per lane are
 * issued before the first store; every byte is read and written once.
 * Asynchronous; EINVAL on misaligned arguments, another loads_per_lane or a
 * copy above 2^31 workgroups. */
lbaxi_status lbaxi_stream_copy(const void* d_src, void* d_dst, size_t bytes, int32_t loads_per_lane,
                               void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBAXI_H */
