/* Host-side driver of both libraries' C ABI for the sanitizer test: every
 * entry point that needs no GPU (descriptor validation, workspace sizing and
 * layout, argument checks, error strings) over valid and invalid inputs.
 * Built with the libraries' host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer; a finding aborts the run.  Prints one line
 * per case and "ok" at the end; exit status 0 when every case gave the
 * status it should. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "lbaxi.h"
#include "lbnn.h"

static int bad = 0;

static int nn_case = 0;  /* 1: report the network library's error text */

static void expect(const char* what, lbaxi_status got, int ok_expected) {
  const int ok = got == LBAXI_OK;
  printf("%-48s status %3d  %s\n", what, (int)got,
         ok ? "" : (nn_case ? lbnn_last_error() : lbaxi_last_error()));
  if (ok != ok_expected) {
    printf("  ^ expected %s\n", ok_expected ? "success" : "an error");
    bad = 1;
  }
}

static lbaxi_side side(int32_t kind) {
  lbaxi_side s;
  memset(&s, 0, sizeof s);
  s.kind = kind;
  s.r_split = -1.0;
  s.kind2 = LBAXI_SIDE_WALL;
  return s;
}

static lbaxi_desc pipe_desc(int32_t nz, int32_t nr, int32_t prec, uint32_t fields) {
  lbaxi_desc d;
  memset(&d, 0, sizeof d);
  d.nz = nz;
  d.nr = nr;
  d.prec = prec;
  d.fields = fields;
  d.tau = 0.8;
  d.rho0 = 1.0;
  d.a0 = 1e-6;
  d.south = side(LBAXI_SIDE_AXIS);
  d.north = side(LBAXI_SIDE_WALL);
  d.west = side(LBAXI_SIDE_PERIODIC);
  d.east = side(LBAXI_SIDE_PERIODIC);
  return d;
}

/* deterministic pseudo-random numbers (64-bit LCG) */
static uint64_t rng = 0x9E3779B97F4A7C15ull;
static int32_t rnd(int32_t lo, int32_t hi) {
  rng = rng * 6364136223846793005ull + 1442695040888963407ull;
  return lo + (int32_t)((rng >> 33) % (uint64_t)(hi - lo + 1));
}

int main(void) {
  size_t b = 0;
  char name[96];
  const uint32_t field_sets[] = {0, LBAXI_SWIRL, LBAXI_SWIRL | LBAXI_THERMAL, LBAXI_MRT,
                                 LBAXI_SWIRL | LBAXI_MRT, LBAXI_ORIGINAL, LBAXI_WET_WALLS,
                                 LBAXI_WET_WALLS | LBAXI_SWIRL | LBAXI_THERMAL, LBAXI_CARTESIAN,
                                 LBAXI_PLANES, LBAXI_PLANES | LBAXI_SWIRL | LBAXI_THERMAL};
  for (int p = 0; p < 3; ++p)
    for (unsigned k = 0; k < sizeof field_sets / sizeof field_sets[0]; ++k) {
      lbaxi_desc d = pipe_desc(37 + 5 * (int)k, 21 + p, p, field_sets[k]);
      snprintf(name, sizeof name, "workspace prec %d fields 0x%x", p, field_sets[k]);
      expect(name, lbaxi_workspace_bytes(1, &d, &b), 1);
    }
  /* a batch of uneven lattices, the largest sizes of the 256-cavity batch */
  lbaxi_desc batch[64];
  for (int k = 0; k < 64; ++k) {
    const int32_t nr = rnd(2, 512);
    batch[k] = pipe_desc(rnd(2, 3 * nr + 2), nr, LBAXI_FP32, LBAXI_SWIRL);
  }
  expect("workspace of 64 uneven lattices", lbaxi_workspace_bytes(64, batch, &b), 1);
  /* row blocks below 4 GiB, planes above it, and the 2^31-element bound */
  lbaxi_desc big = pipe_desc(16384, 7200, LBAXI_FP32, 0);
  expect("workspace 16384 x 7200 FP32 (row blocks)", lbaxi_workspace_bytes(1, &big, &b), 1);
  big.nr = 7300;
  expect("workspace 16384 x 7300 FP32 (planes)", lbaxi_workspace_bytes(1, &big, &b), 1);
  big.fields = LBAXI_PLANES;
  expect("workspace 16384 x 7300 FP32, planes asked", lbaxi_workspace_bytes(1, &big, &b), 1);
  big.nr = 14000;
  big.fields = 0;
  expect("workspace 16384 x 14000 FP64 (below 2^31)", (big.prec = LBAXI_FP64,
         lbaxi_workspace_bytes(1, &big, &b)), 1);
  big.nr = 14600;
  expect("workspace 16384 x 14600 FP64 (above 2^31)", lbaxi_workspace_bytes(1, &big, &b), 0);
  big.prec = LBAXI_FP32;
  big.nr = 1 << 30;
  expect("workspace nr = 2^30", lbaxi_workspace_bytes(1, &big, &b), 0);
  big.nr = 7200;
  big.nz = 0x7fffffff;
  expect("workspace nz = 2^31 - 1", lbaxi_workspace_bytes(1, &big, &b), 0);

  lbaxi_desc d = pipe_desc(1, 8, LBAXI_FP64, 0);
  expect("nz = 1", lbaxi_workspace_bytes(1, &d, &b), 0);
  d = pipe_desc(8, 8, 7, 0);
  expect("unknown precision", lbaxi_workspace_bytes(1, &d, &b), 0);
  d = pipe_desc(8, 8, LBAXI_FP64, 1u << 8);
  expect("unknown field bit", lbaxi_workspace_bytes(1, &d, &b), 0);
  d = pipe_desc(8, 8, LBAXI_FP64, 0);
  d.r0 = 2.0;
  expect("axis with r0 != 0", lbaxi_workspace_bytes(1, &d, &b), 0);
  d = pipe_desc(8, 8, LBAXI_FP64, 0);
  d.east = side(LBAXI_SIDE_WALL);
  expect("periodic on one z-end only", lbaxi_workspace_bytes(1, &d, &b), 0);
  d = pipe_desc(8, 8, LBAXI_FP64, LBAXI_ZOU_HE);
  expect("Zou-He without wet-node walls", lbaxi_workspace_bytes(1, &d, &b), 0);
  lbaxi_desc two[2] = {pipe_desc(8, 8, LBAXI_FP64, 0), pipe_desc(8, 8, LBAXI_FP32, 0)};
  expect("mixed precisions in a batch", lbaxi_workspace_bytes(2, two, &b), 0);
  two[1] = pipe_desc(8, 8, LBAXI_FP64, LBAXI_SWIRL);
  expect("mixed field sets in a batch", lbaxi_workspace_bytes(2, two, &b), 0);
  expect("n = 0", lbaxi_workspace_bytes(0, two, &b), 0);
  expect("NULL descriptors", lbaxi_workspace_bytes(1, NULL, &b), 0);
  expect("NULL size", lbaxi_workspace_bytes(1, two, NULL), 0);

  /* create: argument checks that come before any device call */
  lbaxi_t* h = NULL;
  d = pipe_desc(8, 8, LBAXI_FP64, 0);
  expect("create with NULL out", lbaxi_create(1, &d, NULL, 0, NULL, NULL), 0);
  expect("create with NULL workspace", lbaxi_create(1, &d, NULL, 1 << 20, NULL, &h), 0);
  expect("create with misaligned workspace",
         lbaxi_create(1, &d, (void*)(uintptr_t)0x1004, 1 << 20, NULL, &h), 0);
  expect("create with small workspace", lbaxi_create(1, &d, (void*)(uintptr_t)0x1000, 64, NULL, &h),
         0);
  d.nz = 1;
  expect("create with an invalid descriptor",
         lbaxi_create(1, &d, (void*)(uintptr_t)0x1000, 1 << 20, NULL, &h), 0);
  /* calls on a NULL handle */
  expect("step on NULL", lbaxi_step(NULL, 1), 0);
  expect("residual on NULL", lbaxi_residual(NULL, NULL), 0);
  expect("set_launch on NULL", lbaxi_set_launch(NULL, 64, 1, 0, 0, 1), 0);
  expect("set_fused_walls on NULL", lbaxi_set_fused_walls(NULL, 1), 0);
  lbaxi_destroy(NULL);
  for (int s = -8; s <= 2; ++s)
    if (!lbaxi_strerror((lbaxi_status)s) || !lbaxi_last_error()) bad = 1;
  if (lbaxi_abi_desc_size() != sizeof(lbaxi_desc)) bad = 1;

  /* network: descriptor validation and workspace sizing */
  nn_case = 1;
  lbnn_desc nd;
  memset(&nd, 0, sizeof nd);
  nd.H = 128;
  nd.W = 256;
  nd.c_in = 8;
  nd.c_out = 4;
  nd.max_batch = 4;
  for (int k = 0; k < 4; ++k) nd.widths[k] = 32 << k;
  expect("network workspace 128 x 256", lbnn_workspace_bytes(&nd, &b), 1);
  nd.widths[1] = 48;
  expect("network width not a multiple of 32", lbnn_workspace_bytes(&nd, &b), 0);
  nd.widths[1] = 64;
  nd.max_batch = 128;
  expect("network batch above the 32-bit bound", lbnn_workspace_bytes(&nd, &b), 0);
  nd.max_batch = 4;
  nd.H = 100;
  expect("network height not a multiple of 8", lbnn_workspace_bytes(&nd, &b), 0);
  expect("network NULL descriptor", lbnn_workspace_bytes(NULL, &b), 0);
  lbnn_destroy(NULL);

  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
