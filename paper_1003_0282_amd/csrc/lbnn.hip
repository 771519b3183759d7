// lbnn.hip -- warm-start U-Net for the axisymmetric LB solver: BF16 MFMA
// convolution kernels (forward, backward-data, backward-weight), the glue
// kernels of the U-Net, MSE loss, Adam, and the C ABI of include/lbnn.h.
//
// Every 3x3 convolution is an implicit GEMM on v_mfma_f32_32x32x16_bf16
// (M = pixels, N = output channels, K = 9 taps x input channels): a
// workgroup stages tiles of the shifted input rows and the weight rows in
// LDS and each wave multiplies 32 x 32 blocks out of them; the weight
// gradient stages pixel-major tiles through LDS transposed, since its K is
// the pixel index.  A lane's A fragment is 8 consecutive K of one row (16
// bytes), its B fragment 8 consecutive K of one column.  Any K order shared
// by A and B gives the same sum, so the only layout the code relies on is the
// accumulator's (checked by lbnn_mfma_selftest): register r of lane l holds
// row (r/4)*8 + (l/32)*4 + r%4, column l%32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbnn.h"

typedef unsigned short bf16s;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ inline float bf2f(bf16s h) { return __uint_as_float((unsigned)h << 16); }

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ inline bf16s f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16s)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16s)(u >> 16);
}

// Activation of every 3x3 convolution: softplus, sp(v) = log(1 + e^v).  Its
// derivative, sigmoid(v) = 1 - e^(-sp(v)), follows from the stored output,
// so the backward pass needs no pre-activation.  (A smooth activation keeps
// the gradient of a network with BF16 activations well conditioned: a
// ReLU's mask flips wherever rounding moves a pre-activation across zero.)
// Both use the hardware base-2 exponential and logarithm (__expf, __logf):
// their absolute error, a few 1e-8, is far below the BF16 rounding of the
// stored activations and gradients.
__device__ inline float softplus(float v) {
  return fmaxf(v, 0.0f) + __logf(1.0f + __expf(-fabsf(v)));
}
__device__ inline float softplus_grad(float a) { return 1.0f - __expf(-a); }

__device__ inline f32x16 mfma(u16x8 a, u16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Workgroup b of a grid of G runs on XCD b % 8; map it to tile
// xcd * (G / 8) + b / 8 (the first G % 8 XCDs take one tile more) so that
// neighbouring pixel tiles, which re-read each other's rows for the taps of
// a 3 x 3 convolution, share one L2.  A bijection on [0, G).
__device__ inline int xcd_tile(int b, int G) {
  const int x = b & 7, i = b >> 3, q = G >> 3, rem = G & 7;
  return x < rem ? x * (q + 1) + i : rem * (q + 1) + (x - rem) * q + i;
}

// Row of the 32x32 output block held by accumulator r of a lane in half g.
__device__ inline int acc_row(int r, int g) { return (r >> 2) * 8 + g * 4 + (r & 3); }

// ---------------------------------------------------------------------------
// 3x3 convolution as implicit GEMM.  in [B][H][W][Ck], wt [9][Cn][Ck]
// (K contiguous), out [B][H][W][Cn].  sign = +1: out[p] = sum in[p + off]
// (forward); sign = -1: out[p] = sum in[p - off] (adjoint, gradient of the
// input with wt = the original [9][Ci][Co] weights).
struct ConvArgs {
  const bf16s* in;
  const bf16s* wt;
  const float* bias;  // [Cn] or NULL
  const bf16s* mask;  // [B][H][W][Cn] or NULL: output times softplus_grad(mask)
  bf16s* out;
  int B, H, W, Ck, Cn, sign, act;  // act: softplus on the output
};

// Workgroup tile: PT pixels x NT output channels, 4 waves in a WPX x WCH
// grid, each wave MW x NW blocks of 32 x 32.  K (9 taps x Ck input channels,
// tap-major) is walked in stages of CV_KST: thread t loads row t of the
// stage (a pixel row, shifted by each chunk's tap and zero outside the
// image, or a weight row), eight 16-byte chunks, into LDS (rows padded to
// 144 bytes: conflict-free fragment reads); every wave then reads its
// fragments from LDS and runs 4 MW NW MFMAs while the next stage's loads are
// in flight in registers.  Several taps share a stage when Ck is small.
constexpr int CV_KST = 64;              // flattened K per stage
constexpr int CV_RS = CV_KST + 8;       // LDS row stride (elements)

template <int PT, int NT, int MW, int NW>
__global__ void __launch_bounds__(256) k_conv(ConvArgs A) {
  constexpr int WPX = PT / (32 * MW), WCH = NT / (32 * NW);
  static_assert(WPX * WCH == 4, "4 waves per workgroup");
  constexpr int ROWS = PT + NT, RPT = (ROWS + 255) / 256;  // rows per thread
  constexpr int NCH = CV_KST / 8;                          // chunks per row
  __shared__ __attribute__((aligned(16))) bf16s sa[PT * CV_RS];
  __shared__ __attribute__((aligned(16))) bf16s sb[NT * CV_RS];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, m = l & 31, g = l >> 5;
  const long long npix = (long long)A.B * A.H * A.W;
  const long long pix0 = (long long)xcd_tile(blockIdx.x, gridDim.x) * PT;
  const int n0 = blockIdx.y * NT;
  const long long hw = (long long)A.H * A.W;
  int ln[RPT], ly[RPT], lx[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int row = tid + 256 * k;
    ln[k] = ly[k] = lx[k] = -1;
    const long long p = pix0 + row;
    if (row < PT && p < npix) {
      ln[k] = (int)(p / hw);
      const int rem = (int)(p - (long long)ln[k] * hw);
      ly[k] = rem / A.W;
      lx[k] = rem - ly[k] * A.W;
    }
  }
  const int KT = 9 * A.Ck, S = (KT + CV_KST - 1) / CV_KST;
  u16x8 r[RPT][NCH];
  auto load = [&](int st) {
    const int k0 = st * CV_KST;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int row = tid + 256 * k;
      int t = k0 / A.Ck, c = k0 - t * A.Ck;
#pragma unroll
      for (int q = 0; q < NCH; ++q) {
        r[k][q] = u16x8{};
        if (row < ROWS && t < 9) {
          if (row < PT) {
            const int yy = ly[k] + A.sign * (t / 3 - 1), xx = lx[k] + A.sign * (t % 3 - 1);
            if (ln[k] >= 0 && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
              r[k][q] = *reinterpret_cast<const u16x8*>(
                  A.in + (((long long)ln[k] * A.H + yy) * A.W + xx) * A.Ck + c);
          } else {
            r[k][q] = *reinterpret_cast<const u16x8*>(
                A.wt + ((long long)t * A.Cn + n0 + row - PT) * A.Ck + c);
          }
        }
        c += 8;
        if (c == A.Ck) {
          c = 0;
          ++t;
        }
      }
    }
  };
  f32x16 acc[MW][NW];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[i][j] = f32x16{};
  const int wpx = wave % WPX, wch = wave / WPX;
  load(0);
  for (int st = 0; st < S; ++st) {
    __syncthreads();  // the previous stage's fragments have been read
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int row = tid + 256 * k;
      if (row < ROWS) {
        bf16s* dst = row < PT ? sa + row * CV_RS : sb + (row - PT) * CV_RS;
#pragma unroll
        for (int q = 0; q < NCH; ++q) *reinterpret_cast<u16x8*>(dst + 8 * q) = r[k][q];
      }
    }
    __syncthreads();
    if (st + 1 < S) load(st + 1);
#pragma unroll
    for (int kk = 0; kk < CV_KST / 16; ++kk) {
      if (st * CV_KST + 16 * kk >= KT) break;
      u16x8 af[MW], bf[NW];
#pragma unroll
      for (int i = 0; i < MW; ++i)
        af[i] = *reinterpret_cast<const u16x8*>(sa + ((wpx * MW + i) * 32 + m) * CV_RS + 16 * kk + 8 * g);
#pragma unroll
      for (int j = 0; j < NW; ++j)
        bf[j] = *reinterpret_cast<const u16x8*>(sb + ((wch * NW + j) * 32 + m) * CV_RS + 16 * kk + 8 * g);
#pragma unroll
      for (int i = 0; i < MW; ++i)
#pragma unroll
        for (int j = 0; j < NW; ++j) acc[i][j] = mfma(af[i], bf[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int col = n0 + (wch * NW + j) * 32 + m;
    const float bias = A.bias ? A.bias[col] : 0.0f;
#pragma unroll
    for (int i = 0; i < MW; ++i)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const long long px = pix0 + (wpx * MW + i) * 32 + acc_row(q, g);
        if (px >= npix) continue;
        float v = acc[i][j][q] + bias;
        if (A.act) v = softplus(v);
        const long long o = px * A.Cn + col;
        if (A.mask) v *= softplus_grad(bf2f(A.mask[o]));
        A.out[o] = f2bf(v);
      }
  }
}

// Row-segment variant (W a multiple of TW): the workgroup owns TW pixels of
// one image row x NT output channels.  Per stage of 32 input channels it
// stages the three input rows y - 1 .. y + 1 over x0 - 1 .. x0 + TW (a
// one-pixel halo) and the weights of all nine taps in LDS, so every input
// row is read from memory once per stage instead of once per tap.  The 4
// waves form a (TW / 32) x WCH grid, each owning 32 pixels x NW blocks of 32
// channels, and run 9 taps x 2 K-steps x NW MFMAs per stage.
constexpr int RW_KC = 32;               // input channels per stage (two K-steps of 16)
static_assert(RW_KC == 32, "the weight tile's fragment order assumes 32 channels per stage");
constexpr int RW_RS = RW_KC + 8;        // LDS row stride (elements): 80 bytes

// Which 16-byte piece of the weight tile load f (0 <= f < 9 NT 4) moves:
// tap t, output channel nn, 8-channel chunk q.  Within each run of 64 loads
// (one wave) q is the slowest index, so the 16 lanes that an LDS write
// serves together store 16 channels' chunks side by side (256 contiguous
// bytes) rather than four chunks 512 bytes apart on the same banks; a
// wave's 64 global reads still cover the same 16 whole weight rows.
template <int NT>
__device__ inline void wtile_part(int f, int& t, int& nn, int& q) {
  static_assert(NT % 16 == 0, "runs of 64 loads cover 16 whole output channels");
  t = f / (NT * 4);
  const int rem = f - t * (NT * 4), lo = rem & 63;
  q = lo >> 4;
  nn = (rem >> 6) * 16 + (lo & 15);
}

template <int TW, int NT>
__global__ void __launch_bounds__(256) k_conv_row(ConvArgs A) {
  constexpr int WPX = TW / 32, WCH = 4 / WPX, NW = NT / (32 * WCH);
  static_assert(WPX * WCH == 4 && NW * 32 * WCH == NT, "wave grid");
  constexpr int HX = TW + 2;                      // halo row length (pixels)
  constexpr int NH = 3 * HX * (RW_KC / 8);        // 16-byte loads of the halo
  // the weight loads start on a wave boundary (a multiple of 64 threads)
  constexpr int NHP = (NH + 63) / 64 * 64;
  constexpr int NWT = 9 * NT * (RW_KC / 8);       // 16-byte loads of the weights
  constexpr int LPT = (NHP + NWT + 255) / 256;
  // halo rows sh, then the weights sw, in one buffer that the epilogue
  // reuses for the output tile
  constexpr int SH = 3 * HX * RW_RS;
  __shared__ __attribute__((aligned(16))) bf16s smem[SH + 9 * NT * RW_KC];
  bf16s* const sh = smem;
  // weights in the MFMA's B-fragment order, unpadded: for tap t, block jb of
  // 32 output channels and K-step kk, lane (m, g) reads its 8 channels at
  // ((t * NT / 32 + jb) * 2 + kk) * 512 + (32 g + m) * 8, so a wave's 64
  // 16-byte reads are one contiguous 1 KB (no bank conflicts, no padding)
  bf16s* const sw = smem + SH;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, m = l & 31, g = l >> 5;
  const int wp = wave % WPX, wc = wave / WPX;
  const int segs = A.W / TW;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile % segs, rowi = tile / segs;  // rowi = n * H + y
  const int n = rowi / A.H, y = rowi - n * A.H, x0 = seg * TW;
  const int n0 = blockIdx.y * NT;
  const int S = (A.Ck + RW_KC - 1) / RW_KC;
  u16x8 r[LPT];
  auto load = [&](int st) {
    const int c0 = st * RW_KC;
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int e = tid + 256 * k;
      r[k] = u16x8{};
      if (e < NH) {
        const int hr = e / (HX * 4), rem = e - hr * (HX * 4), hx = rem >> 2, q = rem & 3;
        const int yy = y + hr - 1, xx = x0 + hx - 1, c = c0 + 8 * q;
        if (c < A.Ck && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
          r[k] = *reinterpret_cast<const u16x8*>(
              A.in + (((long long)n * A.H + yy) * A.W + xx) * A.Ck + c);
      } else if (e >= NHP && e < NHP + NWT) {
        int t, nn, q;
        wtile_part<NT>(e - NHP, t, nn, q);
        const int c = c0 + 8 * q;
        if (c < A.Ck)
          r[k] = *reinterpret_cast<const u16x8*>(A.wt + ((long long)t * A.Cn + n0 + nn) * A.Ck + c);
      }
    }
  };
  f32x16 acc[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) acc[j] = f32x16{};
  load(0);
  for (int st = 0; st < S; ++st) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < LPT; ++k) {
      const int e = tid + 256 * k;
      if (e < NH)
        *reinterpret_cast<u16x8*>(sh + (e >> 2) * RW_RS + 8 * (e & 3)) = r[k];
      else if (e >= NHP && e < NHP + NWT) {
        int t, nn, q;
        wtile_part<NT>(e - NHP, t, nn, q);
        *reinterpret_cast<u16x8*>(sw + ((t * (NT / 32) + (nn >> 5)) * 2 + (q >> 1)) * 512 +
                                  ((q & 1) * 32 + (nn & 31)) * 8) = r[k];
      }
    }
    __syncthreads();
    if (st + 1 < S) load(st + 1);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int dy = A.sign * (t / 3 - 1), dx = A.sign * (t % 3 - 1);
      const bf16s* ap = sh + ((1 + dy) * HX + 1 + 32 * wp + m + dx) * RW_RS + 8 * g;
#pragma unroll
      for (int kk = 0; kk < RW_KC / 16; ++kk) {
        if (st * RW_KC + 16 * kk >= A.Ck) break;
        const u16x8 a = *reinterpret_cast<const u16x8*>(ap + 16 * kk);
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          const bf16s* bp = sw + ((t * (NT / 32) + wc * NW + j) * 2 + kk) * 512 + (32 * g + m) * 8;
          acc[j] = mfma(a, *reinterpret_cast<const u16x8*>(bp), acc[j]);
        }
      }
    }
  }
  // Epilogue through LDS: the accumulators, bias and activation applied,
  // go to a TW x NT float tile (row stride NT + 8 floats: the two rows a
  // store instruction writes fall on disjoint halves of the banks); then
  // each thread takes runs of 8 channels of one pixel, applies the mask
  // read as one 16-byte load and stores 16 bytes, so every pixel's NT
  // channels leave as whole lines.  Same float operations per element as
  // storing straight from the accumulators.
  constexpr int OS = NT + 8;
  static_assert(TW * OS * 4 <= (SH + 9 * NT * RW_KC) * 2, "output tile fits the buffer");
  float* const so = reinterpret_cast<float*>(smem);
  __syncthreads();  // every wave has read its last fragments of sh and sw
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int c = (wc * NW + j) * 32 + m;
    const float bias = A.bias ? A.bias[n0 + c] : 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      float v = acc[j][q] + bias;
      if (A.act) v = softplus(v);
      so[(32 * wp + acc_row(q, g)) * OS + c] = v;
    }
  }
  __syncthreads();
  constexpr int RUNS = NT / 8;
  const long long pix0 = (long long)rowi * A.W + x0;
#pragma unroll
  for (int e = tid; e < TW * RUNS; e += 256) {
    const int px = e / RUNS, c8 = e - px * RUNS;
    const float* sp = so + px * OS + 8 * c8;
    const long long o = (pix0 + px) * A.Cn + n0 + 8 * c8;
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = sp[u];
    if (A.mask) {
      const u16x8 mk = *reinterpret_cast<const u16x8*>(A.mask + o);
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] *= softplus_grad(bf2f(mk[u]));
    }
    u16x8 ov;
#pragma unroll
    for (int u = 0; u < 8; ++u) ov[u] = f2bf(v[u]);
    *reinterpret_cast<u16x8*>(A.out + o) = ov;
  }
}

// Weight gradient dW[t][ci][co] += sum_p x[p + off_t][ci] gz[p][co]: for
// each tap a GEMM with M = ci, N = co, K = pixels.  Both operands are stored
// pixel-major (channels contiguous) while the MFMA wants K-contiguous
// fragments, so the pixels are staged through LDS transposed: a loading
// thread reads an 8-pixel x 8-channel block (eight 16-byte loads), transposes
// it in registers and writes eight 16-byte rows [channel][8 pixels]; each
// wave then reads its fragments as single 16-byte LDS reads.
//
// Workgroup: 4 waves, one tap, a (32 MB) ci x (32 NB) co tile, a chunk of
// pixels walked in stages of SP = wg_sp(MB, NB) pixels (SP / 16 K-steps, as
// many as the 256 threads can load in one round); wave w owns block
// (w % MB, (w / MB) % NB) and the K-steps kk with kk % KS = w / (MB NB),
// KS = 4 / (MB NB).  Each workgroup stores its partial sums in the slice
// of its pixel chunk, part[chunk] = {dW [9][Ci][Co], db [Co]}; k_sum_chunks
// then adds the slices in chunk order, so the result does not depend on
// which workgroup finishes first (no atomics: training repeats bit for
// bit).  The bias gradient db[co] = sum_p gz[p][co] comes from the
// workgroups of the centre tap and the first ci block, whose gz loads
// cover every pixel of their chunk once: their loading threads add up what
// they load, and the sums meet in LDS in a fixed order.  x has Cx channels
// (the padded input of the first layer); only ci < Ci are written.
struct WgradArgs {
  const bf16s* x;   // [B][H][W][Cx]
  const bf16s* gz;  // [B][H][W][Co]
  float* part;      // [chunks][9 Ci Co + Co]
  int B, H, W, Cx, Ci, Co, chunk;
  int cib, cob;     // ci / co tiles per tap
};

// Pixels per stage: the x and g tiles take (MB + NB) SP / 2 loading threads.
__host__ __device__ constexpr int wg_sp(int mb, int nb) { return mb + nb == 2 ? 256 : 128; }

// Pixel q = p0 + k of a stage, walked incrementally: (n, y, x).
struct PixCursor {
  int n, y, x;
};
__device__ inline PixCursor pix_at(long long p, int H, int W) {
  const long long hw = (long long)H * W;
  PixCursor c;
  c.n = (int)(p / hw);
  const int rem = (int)(p - (long long)c.n * hw);
  c.y = rem / W;
  c.x = rem - c.y * W;
  return c;
}
__device__ inline void pix_next(PixCursor& c, int H, int W) {
  if (++c.x == W) {
    c.x = 0;
    if (++c.y == H) {
      c.y = 0;
      ++c.n;
    }
  }
}

// 8 x 8 transpose of 16-bit elements: out[j][k] = in[k][j].
__device__ inline void transpose8(const u16x8* in, u16x8* out) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int k = 0; k < 8; ++k) out[j][k] = in[k][j];
}

template <int MB, int NB>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs A) {
  constexpr int KS = 4 / (MB * NB);
  constexpr int WG_SP = wg_sp(MB, NB);
  constexpr int WG_RS = WG_SP + 8;          // LDS row stride: an odd multiple of 16 bytes
  constexpr int XT = 4 * MB * (WG_SP / 8);  // loading threads of the x tile (8 px x 8 ch each)
  constexpr int GT = 4 * NB * (WG_SP / 8);
  static_assert(XT + GT <= 256, "one load round per stage");
  __shared__ __attribute__((aligned(16))) bf16s sx[32 * MB * WG_RS];
  __shared__ __attribute__((aligned(16))) bf16s sg[32 * NB * WG_RS];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, m = l & 31, g = l >> 5;
  int blk = blockIdx.y;
  const int t = blk % 9;
  blk /= 9;
  const int ci0 = (blk % A.cib) * 32 * MB, co0 = (blk / A.cib) * 32 * NB;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  const long long npix = (long long)A.B * A.H * A.W;
  const int cidx = xcd_tile(blockIdx.x, gridDim.x);
  const long long p_beg = (long long)cidx * A.chunk;
  const long long p_end = std::min<long long>(p_beg + A.chunk, npix);
  // this thread's loading role: an 8-pixel group and an 8-channel group
  const bool ldx = tid < XT, ldg = tid >= XT && tid < XT + GT;
  const int lt = ldx ? tid : tid - XT;
  const int pg = lt % (WG_SP / 8), cg = lt / (WG_SP / 8);
  const int mb = wave % MB, nb = (wave / MB) % NB, ks = wave / (MB * NB);
  const bool bias_wg = t == 4 && ci0 == 0;  // workgroup-uniform
  float bs[8] = {};
  u16x8 r[8];
  auto load = [&](long long p0) {
    const u16x8 zero = {};
    if (!ldx && !ldg) return;
    long long p = p0 + 8 * pg;
    PixCursor c = pix_at(p < npix ? p : 0, A.H, A.W);
#pragma unroll
    for (int k = 0; k < 8; ++k, ++p) {
      r[k] = zero;
      if (p < p_end) {
        if (ldx) {
          const int ch = ci0 + 8 * cg, yy = c.y + dy, xx = c.x + dx;
          if (ch < A.Cx && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
            r[k] = *reinterpret_cast<const u16x8*>(
                A.x + (((long long)c.n * A.H + yy) * A.W + xx) * A.Cx + ch);
        } else {
          r[k] = *reinterpret_cast<const u16x8*>(A.gz + p * A.Co + co0 + 8 * cg);
        }
      }
      pix_next(c, A.H, A.W);
    }
  };
  f32x16 acc = {};
  load(p_beg);
  for (long long p0 = p_beg; p0 < p_end; p0 += WG_SP) {
    __syncthreads();  // the previous stage's fragments have been read
    if (bias_wg && ldg) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int e = 0; e < 8; ++e) bs[e] += bf2f(r[k][e]);
    }
    if (ldx || ldg) {
      u16x8 tr[8];
      transpose8(r, tr);
      bf16s* base = (ldx ? sx : sg) + (8 * cg) * WG_RS + 8 * pg;
#pragma unroll
      for (int j = 0; j < 8; ++j) *reinterpret_cast<u16x8*>(base + j * WG_RS) = tr[j];
    }
    __syncthreads();
    if (p0 + WG_SP < p_end) load(p0 + WG_SP);  // next stage in flight during the MFMAs
#pragma unroll
    for (int kk = 0; kk < WG_SP / 16; ++kk) {
      if (kk % KS != ks) continue;
      const u16x8 a = *reinterpret_cast<const u16x8*>(sx + (32 * mb + m) * WG_RS + 16 * kk + 8 * g);
      const u16x8 b = *reinterpret_cast<const u16x8*>(sg + (32 * nb + m) * WG_RS + 16 * kk + 8 * g);
      acc = mfma(a, b, acc);
    }
  }
  float* part = A.part + (long long)cidx * (9LL * A.Ci * A.Co + A.Co);
  if (bias_wg) {
    // the gz loaders' column sums, pixel groups added in order
    constexpr int PG = WG_SP / 8;
    static_assert(sizeof(sg) >= 32 * NB * PG * sizeof(float), "bias reduction buffer");
    float* red = reinterpret_cast<float*>(sg);
    __syncthreads();  // every wave is done with the staged tiles
    if (ldg) {
#pragma unroll
      for (int e = 0; e < 8; ++e) red[(8 * cg + e) * PG + pg] = bs[e];
    }
    __syncthreads();
    if (tid < 32 * NB) {
      float b = 0.0f;
      for (int k = 0; k < PG; ++k) b += red[tid * PG + k];
      part[9LL * A.Ci * A.Co + co0 + tid] = b;
    }
  }
  // the KS waves that split this block's K-steps meet in LDS (fixed order)
  const int co = co0 + 32 * nb + m;
  if (KS == 1) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int ci = ci0 + 32 * mb + acc_row(q, g);
      if (ci < A.Ci) part[((long long)t * A.Ci + ci) * A.Co + co] = acc[q];
    }
  } else {
    // waves ks > 0 hand their sums to wave ks = 0 of the same block through
    // LDS (the x tile is no longer needed), which adds them in ks order
    constexpr int L = 64 * MB * NB;  // threads of one K-step slice
    static_assert(sizeof(sx) >= 16 * (KS - 1) * L * sizeof(float), "reduction buffer");
    float* red = reinterpret_cast<float*>(sx);
    const int lt = tid % L;
    __syncthreads();  // every wave is done with the staged tiles
    if (ks > 0) {
#pragma unroll
      for (int q = 0; q < 16; ++q) red[(q * (KS - 1) + ks - 1) * L + lt] = acc[q];
    }
    __syncthreads();
    if (ks == 0) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        float v = acc[q];
        for (int k = 1; k < KS; ++k) v += red[(q * (KS - 1) + k - 1) * L + lt];
        const int ci = ci0 + 32 * mb + acc_row(q, g);
        if (ci < A.Ci) part[((long long)t * A.Ci + ci) * A.Co + co] = v;
      }
    }
  }
}

// Row-segment weight gradient (W a multiple of WR_TW): a workgroup owns a
// 32 ci x 32 co tile and a run of row segments of WR_TW pixels.  Per segment
// it stages, transposed to [channel][pixel] (8 x 8 register transposes, rows
// padded to an odd multiple of 16 bytes), the three input rows y - 1 .. y + 1
// over x0 - 8 .. x0 + WR_TW + 7 (zero outside the image) and the gradient row
// y over x0 .. x0 + WR_TW - 1; all nine taps then read the same staged rows,
// the tap's x shift being an offset into the row (one 16-byte LDS read for
// dx = 0, eight 2-byte reads otherwise).  Wave w owns the taps t = w mod 4
// over all WR_TW / 16 K-steps.  Partial sums per chunk of segments, the
// bias gradient from the workgroups of the first ci block, as in k_wgrad.
constexpr int WR_TW = 128;                 // pixels per row segment
constexpr int WR_XS = WR_TW + 16 + 8;      // x row: 8-pixel pads each side + 8 (152 el.)
constexpr int WR_GS = WR_TW + 8;           // g row stride (136 elements)

__global__ void __launch_bounds__(256) k_wgrad_row(WgradArgs A) {
  constexpr int XG = WR_TW / 8 + 2;            // 8-pixel groups of an x row (with pads)
  constexpr int NXB = 3 * XG * 4;              // 8 x 8 blocks of the x rows (32 ci)
  constexpr int NGB = (WR_TW / 8) * 4;         // 8 x 8 blocks of the g row (32 co)
  __shared__ __attribute__((aligned(16))) bf16s sx[3 * 32 * WR_XS];
  __shared__ __attribute__((aligned(16))) bf16s sg[32 * WR_GS];
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, m = l & 31, g = l >> 5;
  const int blk = blockIdx.y;
  const int ci0 = (blk % A.cib) * 32, co0 = (blk / A.cib) * 32;
  const int segs = A.W / WR_TW;
  const long long nseg = (long long)A.B * A.H * segs;
  const int cidx = xcd_tile(blockIdx.x, gridDim.x);
  const long long s_beg = (long long)cidx * A.chunk;
  const long long s_end = std::min<long long>(s_beg + A.chunk, nseg);
  f32x16 acc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[k] = f32x16{};
  static_assert(NXB < 256 && NGB <= 256 && NXB + NGB <= 512, "two load rounds");
  const bool bias_wg = ci0 == 0;  // workgroup-uniform
  float bs[8] = {};
  const u16x8 zero = {};
  for (long long sgi = s_beg; sgi < s_end; ++sgi) {
    const int seg = (int)(sgi % segs);
    const long long rowi = sgi / segs;
    const int n = (int)(rowi / A.H), y = (int)(rowi - (long long)n * A.H), x0 = seg * WR_TW;
    __syncthreads();  // the previous segment's fragments have been read
    for (int b = tid; b < NXB + NGB; b += 256) {
      u16x8 v[8], tv[8];
      if (b < NXB) {
        const int hr = b / (XG * 4), rem = b - hr * (XG * 4), xg = rem >> 2, cg = rem & 3;
        const int yy = y + hr - 1, ch = ci0 + 8 * cg;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int xx = x0 - 8 + 8 * xg + k;
          v[k] = (ch < A.Cx && yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
                     ? *reinterpret_cast<const u16x8*>(
                           A.x + (((long long)n * A.H + yy) * A.W + xx) * A.Cx + ch)
                     : zero;
        }
        transpose8(v, tv);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<u16x8*>(sx + (hr * 32 + 8 * cg + j) * WR_XS + 8 * xg) = tv[j];
      } else {
        const int f = b - NXB, xg = f >> 2, cg = f & 3;
        const long long p = rowi * A.W + x0 + 8 * xg;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          v[k] = *reinterpret_cast<const u16x8*>(A.gz + (p + k) * A.Co + co0 + 8 * cg);
        if (bias_wg) {
#pragma unroll
          for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) bs[e] += bf2f(v[k][e]);
        }
        transpose8(v, tv);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          *reinterpret_cast<u16x8*>(sg + (8 * cg + j) * WR_GS + 8 * xg) = tv[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < WR_TW / 16; ++kk) {
      const u16x8 bfr = *reinterpret_cast<const u16x8*>(sg + m * WR_GS + 16 * kk + 8 * g);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int t = wave + 4 * k;
        if (t >= 9) break;
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        const bf16s* ap = sx + ((1 + dy) * 32 + m) * WR_XS + 8 + 16 * kk + 8 * g + dx;
        u16x8 afr;
        if (dx == 0) {
          afr = *reinterpret_cast<const u16x8*>(ap);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) afr[e] = ap[e];
        }
        acc[k] = mfma(afr, bfr, acc[k]);
      }
    }
  }
  float* part = A.part + (long long)cidx * (9LL * A.Ci * A.Co + A.Co);
  if (bias_wg) {
    // thread tid loaded gz block b = tid or tid + 256 (if in the gz range);
    // its column sums meet in LDS, pixel groups added in order
    constexpr int PG = WR_TW / 8;
    static_assert(sizeof(sg) >= 32 * PG * sizeof(float), "bias reduction buffer");
    float* red = reinterpret_cast<float*>(sg);
    __syncthreads();  // every wave is done with the staged tiles
    const int b = tid >= NXB ? tid : tid + 256;
    if (b < NXB + NGB) {
      const int f = b - NXB, xg = f >> 2, cg = f & 3;
#pragma unroll
      for (int e = 0; e < 8; ++e) red[(8 * cg + e) * PG + xg] = bs[e];
    }
    __syncthreads();
    if (tid < 32) {
      float bsum = 0.0f;
      for (int k = 0; k < PG; ++k) bsum += red[tid * PG + k];
      part[9LL * A.Ci * A.Co + co0 + tid] = bsum;
    }
  }
  const int co = co0 + m;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int t = wave + 4 * k;
    if (t >= 9) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int ci = ci0 + acc_row(q, g);
      if (ci < A.Ci) part[((long long)t * A.Ci + ci) * A.Co + co] = acc[k][q];
    }
  }
}

// out[w] = sum over chunks of part[c][w] in a fixed order: the second pass
// of every parameter-gradient reduction.  The chunks are cut into G
// contiguous runs (a workgroup covers 256 / G elements); thread (run,
// element) adds its run in chunk order with eight loads in flight, then the
// G run sums are added in run order.  Several runs keep the dependent chain
// of loads short where there are many chunks and few elements.
template <int G>
__global__ void __launch_bounds__(256) k_sum_chunks(const float* part, float* out, long long n,
                                                    int nchunk) {
  constexpr int E = 256 / G;
  __shared__ float red[256];
  const int e = threadIdx.x % E, run = threadIdx.x / E;
  const long long w = (long long)blockIdx.x * E + e;
  const int len = (nchunk + G - 1) / G;
  const int c1 = min(nchunk, (run + 1) * len);
  float s = 0.0f;
  if (w < n) {
    int c = run * len;
    for (; c + 8 <= c1; c += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(long long)(c + u) * n + w];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < c1; ++c) s += part[(long long)c * n + w];
  }
  if (G == 1) {
    if (w < n) out[w] = s;
    return;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (run == 0 && w < n) {
    float t = red[e];
    for (int k = 1; k < G; ++k) t += red[k * E + e];
    out[w] = t;
  }
}

// The same for FP64 partial sums reduced to one value by one workgroup:
// thread t adds the partials t, t + 256, ... in order, then a fixed tree.
__global__ void __launch_bounds__(256) k_sum_chunks_d(const double* part, double* out,
                                                      int nchunk) {
  __shared__ double red[256];
  double s = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) s += part[c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ---- U-Net glue --------------------------------------------------------------

// FP32 [B][H][W][c_in] -> BF16 [B][H][W][16], zero channels beyond c_in.
__global__ void k_input(const float* x, bf16s* out, long long npix, int c_in) {
  const unsigned p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  u16x8 o[2];
#pragma unroll
  for (int c = 0; c < 16; ++c) o[c >> 3][c & 7] = c < c_in ? f2bf(x[(long long)p * c_in + c]) : (bf16s)0;
  *reinterpret_cast<u16x8*>(out + 16LL * p) = o[0];
  *reinterpret_cast<u16x8*>(out + 16LL * p + 8) = o[1];
}

// The glue kernels below move 8 channels (16 bytes) per thread and index
// with 32-bit arithmetic (the plan bounds every tensor below 2^31 vectors).

// 2x2 average pooling: out [B][H/2][W/2][C].
__global__ void k_pool(const bf16s* in, bf16s* out, int B, int H, int W, int C) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned G = C / 8, h = H / 2, w = W / 2;
  if (v >= (unsigned)B * h * w * G) return;
  const unsigned cg = v % G, q = v / G, x = q % w, r = q / w, y = r % h, n = r / h;
  const long long b = (((long long)n * H + 2 * y) * W + 2 * x) * C + 8 * cg;
  const u16x8 a = *reinterpret_cast<const u16x8*>(in + b);
  const u16x8 c = *reinterpret_cast<const u16x8*>(in + b + C);
  const u16x8 d = *reinterpret_cast<const u16x8*>(in + b + (long long)W * C);
  const u16x8 e = *reinterpret_cast<const u16x8*>(in + b + (long long)W * C + C);
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = f2bf(0.25f * (bf2f(a[k]) + bf2f(c[k]) + bf2f(d[k]) + bf2f(e[k])));
  *reinterpret_cast<u16x8*>(out + 8LL * v) = o;
}

// Gradient into the pre-activation of an encoder output e [B][H][W][C]: a
// quarter of the pooled gradient of its 2x2 parent plus the skip gradient,
// times the activation's derivative softplus_grad(e).
__global__ void k_pool_back(const bf16s* gp, const bf16s* gskip, const bf16s* e, bf16s* ge,
                            int B, int H, int W, int C) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned G = C / 8;
  if (v >= (unsigned)B * H * W * G) return;
  const unsigned cg = v % G, q = v / G, x = q % W, r = q / W, y = r % H, n = r / H;
  const u16x8 pg = *reinterpret_cast<const u16x8*>(
      gp + (((long long)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + 8 * cg);
  const u16x8 sk = *reinterpret_cast<const u16x8*>(gskip + 8LL * v);
  const u16x8 ev = *reinterpret_cast<const u16x8*>(e + 8LL * v);
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float t = 0.25f * bf2f(pg[k]) + bf2f(sk[k]);
    o[k] = f2bf(t * softplus_grad(bf2f(ev[k])));
  }
  *reinterpret_cast<u16x8*>(ge + 8LL * v) = o;
}

// cat [B][H][W][Cu + Cs] = (nearest 2x upsample of u [B][H/2][W/2][Cu], s).
__global__ void k_upcat(const bf16s* u, const bf16s* s, bf16s* cat, int B, int H, int W, int Cu,
                        int Cs) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned G = (Cu + Cs) / 8, Gu = Cu / 8;
  if (v >= (unsigned)B * H * W * G) return;
  const unsigned cg = v % G, p = v / G;
  u16x8 o;
  if (cg >= Gu) {
    o = *reinterpret_cast<const u16x8*>(s + (long long)p * Cs + 8 * (cg - Gu));
  } else {
    const unsigned x = p % W, r = p / W, y = r % H, n = r / H;
    o = *reinterpret_cast<const u16x8*>(u + (((long long)n * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu +
                                        8 * cg);
  }
  *reinterpret_cast<u16x8*>(cat + 8LL * v) = o;
}

// Backward of k_upcat: gu [B][H/2][W/2][Cu] = sum of the 2x2 children times
// softplus_grad(u) (u is an activation output; gu is the gradient of its
// pre-activation); the skip
// part is copied to gskip [B][H][W][Cs].  Threads [0, nu) cover gu, the next
// ns threads gskip (8 channels each).
__global__ void k_upcat_back(const bf16s* gcat, const bf16s* u, bf16s* gu, bf16s* gskip, int B,
                             int H, int W, int Cu, int Cs) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = Cu + Cs;
  const unsigned h = H / 2, w = W / 2, Gu = Cu / 8, Gs = Cs / 8;
  const unsigned nu = (unsigned)B * h * w * Gu, ns = (unsigned)B * H * W * Gs;
  if (v < nu) {
    const unsigned cg = v % Gu, q = v / Gu, x = q % w, r = q / w, y = r % h, n = r / h;
    const long long b = (((long long)n * H + 2 * y) * W + 2 * x) * C + 8 * cg;
    const u16x8 a = *reinterpret_cast<const u16x8*>(gcat + b);
    const u16x8 c = *reinterpret_cast<const u16x8*>(gcat + b + C);
    const u16x8 d = *reinterpret_cast<const u16x8*>(gcat + b + (long long)W * C);
    const u16x8 e = *reinterpret_cast<const u16x8*>(gcat + b + (long long)W * C + C);
    const u16x8 uv = *reinterpret_cast<const u16x8*>(u + 8LL * v);
    u16x8 o;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float t = bf2f(a[k]) + bf2f(c[k]) + bf2f(d[k]) + bf2f(e[k]);
      o[k] = f2bf(t * softplus_grad(bf2f(uv[k])));
    }
    *reinterpret_cast<u16x8*>(gu + 8LL * v) = o;
  } else if (v < nu + ns) {
    const unsigned j = v - nu, cg = j % Gs, p = j / Gs;
    *reinterpret_cast<u16x8*>(gskip + 8LL * j) =
        *reinterpret_cast<const u16x8*>(gcat + (long long)p * C + Cu + 8 * cg);
  }
}

// Head: y[p][k] = sum_c d0[p][c] Wh[c][k] + bh[k] (FP32 parameters, K <= 8,
// C a multiple of 8: the row of d0 is read 16 bytes at a time).  With a
// target: gy = 2 (y - t) / N into gy and the workgroup's squared error into
// loss_part[block] (added in block order by k_sum_chunks_d).
__global__ void __launch_bounds__(256) k_head(const bf16s* d0, const float* Wh, const float* bh,
                                              float* y, const float* tgt, float* gy,
                                              double* loss_part, long long npix, int C, int K,
                                              double inv_n) {
  __shared__ float red[256];
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float se = 0.0f;
  if (p < npix) {
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = k < K ? bh[k] : 0.0f;
    for (int c0 = 0; c0 < C; c0 += 8) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(d0 + p * C + c0);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float d = bf2f(v[e]);
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < K) acc[k] += d * Wh[(c0 + e) * K + k];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= K) break;
      y[p * K + k] = acc[k];
      if (tgt) {
        const float dlt = acc[k] - tgt[p * K + k];
        se += dlt * dlt;
        gy[p * K + k] = (float)(2.0 * inv_n) * dlt;
      }
    }
  }
  if (!tgt) return;
  red[threadIdx.x] = se;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = (double)red[0];
}

// Head backward, input side: gd0[p][c] = (sum_k gy[p][k] Wh[c][k])
// times softplus_grad(d0) (d0 is an activation output); 8 channels per
// 16-byte load and store.
__global__ void __launch_bounds__(256) k_head_back(const bf16s* d0, const float* gy,
                                                   const float* Wh, bf16s* gd0, long long npix,
                                                   int C, int K) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float g[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) g[k] = k < K ? gy[p * K + k] : 0.0f;
  for (int c0 = 0; c0 < C; c0 += 8) {
    const u16x8 v = *reinterpret_cast<const u16x8*>(d0 + p * C + c0);
    u16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float s = 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < K) s += g[k] * Wh[(c0 + e) * K + k];
      o[e] = f2bf(s * softplus_grad(bf2f(v[e])));
    }
    *reinterpret_cast<u16x8*>(gd0 + p * C + c0) = o;
  }
}

// Head backward, parameter side: dWh[c][k] = sum_p d0[p][c] gy[p][k] and
// dbh[k] = sum_p gy[p][k].  Thread t owns channels 8 (t % G) .. + 7
// (G = C / 8, one 16-byte load of d0 per pixel) and every (256 / G)-th
// pixel of a chunk of 64 (256 / G) pixels, accumulating 8 x K products in
// registers; the partial sums meet in LDS in a fixed order and the chunk's
// C K + K sums go to part[chunk] (dWh then dbh), which k_sum_chunks adds.
// C <= 256 a multiple of 8, K <= 8.
__global__ void __launch_bounds__(256) k_head_wgrad(const bf16s* d0, const float* gy, float* part,
                                                    long long npix, int C, int K) {
  __shared__ float red[8 * 256 * 8];  // [k][thread][e]
  __shared__ float redb[256 * 8];     // [thread][k]
  const int G = C / 8, nq = 256 / G;
  const int cg = threadIdx.x % G, q = threadIdx.x / G;
  const long long chunk = 64LL * nq;
  const long long p0 = (long long)blockIdx.x * chunk;
  const long long p1 = std::min<long long>(p0 + chunk, npix);
  float s[8][8] = {}, sb[8] = {};
  if (q < nq)
    for (long long p = p0 + q; p < p1; p += nq) {
      const u16x8 v = *reinterpret_cast<const u16x8*>(d0 + p * C + 8 * cg);
      float gk[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) gk[k] = k < K ? gy[p * K + k] : 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        sb[k] += gk[k];
#pragma unroll
        for (int e = 0; e < 8; ++e) s[k][e] += bf2f(v[e]) * gk[k];
      }
    }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) red[(k * 256 + threadIdx.x) * 8 + e] = s[k][e];
    redb[threadIdx.x * 8 + k] = cg == 0 ? sb[k] : 0.0f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < C * K + K; t += 256) {
    float acc = 0.0f;
    if (t < C * K) {
      const int c = t / K, k = t % K, g = c / 8, e = c % 8;
      for (int j = 0; j < nq; ++j) acc += red[(k * 256 + j * G + g) * 8 + e];
    } else {
      const int k = t - C * K;
      for (int j = 0; j < nq; ++j) acc += redb[(j * G) * 8 + k];
    }
    part[(long long)blockIdx.x * (C * K + K) + t] = acc;
  }
}

// FP32 master W [9][ci][co] -> BF16 copies wf [9][co][Ck] (forward) and
// wb [9][Ck][co] (adjoint), input channels zero-padded to Ck.
__global__ void k_cast_w(const float* W, bf16s* wf, bf16s* wb, int ci, int Ck, int co) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = 9LL * Ck * co;
  if (k >= total) return;
  const int o = (int)(k % co);
  const int c = (int)((k / co) % Ck);
  const int t = (int)(k / ((long long)co * Ck));
  const bf16s v = c < ci ? f2bf(W[((long long)t * ci + c) * co + o]) : (bf16s)0;
  wb[k] = v;
  wf[((long long)t * co + o) * Ck + c] = v;
}

// The convolution weights' place in the parameter vector and their BF16
// copies, for the Adam step to refresh the copies as it updates.
constexpr int MAXCONV = 14;
struct WCopies {
  long long off[MAXCONV];  // first weight of convolution q ([9][ci][co])
  int ci[MAXCONV], Ck[MAXCONV], co[MAXCONV];
  bf16s* wf[MAXCONV];
  bf16s* wb[MAXCONV];
};

// Adam step of every parameter.  A convolution weight is also written to
// its BF16 copies (the value k_cast_w would write), so a step needs no cast
// pass; the zero-padded input channels of the copies are left as they are.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float eps, float c1, float c2, WCopies W) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  const float pk = p[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  p[k] = pk;
  // which convolution's weights k is, if any (constant indices only)
  long long rel = -1;
  int ci = 1, Ck = 1, co = 1;
  bf16s *wf = nullptr, *wb = nullptr;
#pragma unroll
  for (int q = 0; q < MAXCONV; ++q)
    if (k >= W.off[q] && k < W.off[q] + 9LL * W.ci[q] * W.co[q]) {
      rel = k - W.off[q];
      ci = W.ci[q];
      Ck = W.Ck[q];
      co = W.co[q];
      wf = W.wf[q];
      wb = W.wb[q];
    }
  if (rel >= 0) {
    const int o = (int)(rel % co), c = (int)((rel / co) % ci), t = (int)(rel / ((long long)co * ci));
    const bf16s b = f2bf(pk);
    wb[((long long)t * Ck + c) * co + o] = b;
    wf[((long long)t * co + o) * Ck + c] = b;
  }
}

__global__ void k_zero(float* p, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.0f;
}

__global__ void k_set_i32(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

struct FieldOut {
  float* p[8];
  float sc[8], of[8];
};

// y [B][H][W][K] -> fields; smooth: separable (1, 2, 1)/4 along H and W with
// the edge value repeated.
__global__ void k_to_fields(const float* y, int B, int H, int W, int K, int smooth, FieldOut o) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long hw = (long long)H * W;
  if (p >= (long long)B * hw) return;
  const int n = (int)(p / hw);
  const int rem = (int)(p - (long long)n * hw);
  const int r = rem / W, c = rem - (rem / W) * W;
  for (int k = 0; k < K; ++k) {
    if (!o.p[k]) continue;
    float v;
    if (smooth) {
      v = 0.0f;
      for (int dr = -1; dr <= 1; ++dr) {
        const int rr = min(max(r + dr, 0), H - 1);
        const float wr = dr == 0 ? 0.5f : 0.25f;
        for (int dc = -1; dc <= 1; ++dc) {
          const int cc = min(max(c + dc, 0), W - 1);
          const float wc = dc == 0 ? 0.5f : 0.25f;
          v += wr * wc * y[(((long long)n * H + rr) * W + cc) * K + k];
        }
      }
    } else {
      v = y[p * K + k];
    }
    o.p[k][p] = v * o.sc[k] + o.of[k];
  }
}

// Layout self-test: A[i][k] = (i + 2k) mod 7 - 3, B[k][j] = (3k + j) mod 5 - 2
// (exact in BF16, exact FP32 sums); each lane checks its 16 accumulators.
__global__ void k_mfma_selftest(int* bad) {
  const int l = threadIdx.x, m = l & 31, g = l >> 5;
  u16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 8 * g + e;
    a[e] = f2bf((float)((m + 2 * k) % 7 - 3));
    b[e] = f2bf((float)((3 * k + m) % 5 - 2));
  }
  f32x16 acc = {};
  acc = mfma(a, b, acc);
  int nb = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = acc_row(r, g), j = m;
    float s = 0.0f;
    for (int k = 0; k < 16; ++k) s += (float)((i + 2 * k) % 7 - 3) * (float)((3 * k + j) % 5 - 2);
    if (acc[r] != s) ++nb;
  }
  if (nb) atomicAdd(bad, nb);
}

// ============================================================================
// host side
// ============================================================================

namespace {

thread_local std::string g_nerr = "no error";
lbaxi_status nfail(lbaxi_status s, const std::string& m) {
  g_nerr = m;
  return s;
}
#define NCHK(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return nfail(LBAXI_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct Conv {
  int ci, Ck, co;         // real / padded input channels, output channels
  long long off_W, off_b; // offsets in the flat FP32 parameter vector
  size_t wf, wb;          // byte offsets of the BF16 copies in the workspace
};

enum { E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B, NCONV };
static_assert(NCONV == MAXCONV, "one weight-copy entry per convolution");

struct Plan {
  lbnn_desc d;
  Conv cv[NCONV];
  long long off_hW, off_hb, nparam;
  // workspace byte offsets
  size_t params, grads, m1, m2, wcopies, loss, act, part, loss_part, total;
  // activations (BF16) per level, element counts per sample
  size_t xin, e_a[4], e_b[4], pool[3], cat[3], d_a[3], d_b[3], y, gy, gbig1[4], gbig2[4],
      gcat[3], gskip[3];
};

long long npix_lvl(const lbnn_desc& d, int l) { return (long long)(d.H >> l) * (d.W >> l); }

unsigned blocks(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Level (image size H >> lvl) of convolution k of the U-Net.
int conv_level(int k) { return k < D2A ? k / 2 : 2 - (k - D2A) / 2; }

// Launch shape of the weight gradient of a convolution with padded input
// channels Ck, real ci and co outputs on a B x H x W level: the row-segment
// kernel (narrow outputs on rows a multiple of WR_TW wide) or the tiled one,
// its pixel (segment) chunk, and the grid: gx chunks x gy tiles.
struct WgShape {
  bool row;
  int MB, NB, cib, cob, chunk;
  long long gx, gy;
};

WgShape wgrad_shape(int Ck, int co, int B, int H, int W) {
  WgShape S;
  const long long npix = (long long)B * H * W;
  S.row = W % WR_TW == 0 && co % 64 != 0;
  if (S.row) {
    S.MB = S.NB = 1;
    S.cib = (Ck + 31) / 32;
    S.cob = co / 32;
    const long long nseg = (long long)B * H * (W / WR_TW);
    const long long tiles = (long long)S.cib * S.cob;
    // about 512 workgroups, each at least 4 segments long (fewer chunks:
    // less partial-sum traffic for the fixed-order reduction)
    S.chunk = (int)std::max<long long>(4, (nseg * tiles + 511) / 512);
    S.gx = (nseg + S.chunk - 1) / S.chunk;
    S.gy = tiles;
  } else {
    S.MB = Ck >= 64 && Ck % 64 == 0 ? 2 : 1;
    S.NB = co % 64 == 0 ? 2 : 1;
    S.cib = (Ck + 32 * S.MB - 1) / (32 * S.MB);
    S.cob = co / (32 * S.NB);
    const long long tiles = 9LL * S.cib * S.cob;
    // about 1024 workgroups, each at least one and at most 64 stages long
    const int sp = wg_sp(S.MB, S.NB);
    long long ch = (npix * tiles + 1023) / 1024;
    ch = std::max<long long>(sp, std::min<long long>(64LL * sp, ch));
    S.chunk = (int)((ch + sp - 1) / sp * sp);
    S.gx = blocks(npix, S.chunk);
    S.gy = tiles;
  }
  return S;
}

// Pixel chunks of the head's parameter gradient.
long long head_chunks(long long npix, int C) { return blocks(npix, 64 * (256 / (C / 8))); }

bool plan(const lbnn_desc& d, Plan& P) {
  P.d = d;
  const int c0 = d.widths[0], c1 = d.widths[1], c2 = d.widths[2], c3 = d.widths[3];
  const int io[NCONV][2] = {{d.c_in, c0}, {c0, c0}, {c0, c1}, {c1, c1}, {c1, c2},
                            {c2, c2},     {c2, c3}, {c3, c3}, {c3 + c2, c2}, {c2, c2},
                            {c2 + c1, c1}, {c1, c1}, {c1 + c0, c0}, {c0, c0}};
  long long off = 0;
  for (int k = 0; k < NCONV; ++k) {
    Conv& c = P.cv[k];
    c.ci = io[k][0];
    c.Ck = k == E0A ? 16 : io[k][0];
    c.co = io[k][1];
    c.off_W = off;
    off += 9LL * c.ci * c.co;
    c.off_b = off;
    off += c.co;
  }
  P.off_hW = off;
  off += (long long)c0 * d.c_out;
  P.off_hb = off;
  off += d.c_out;
  P.nparam = off;
  size_t o = 0;
  P.params = o; o = al(o + 4 * (size_t)P.nparam);
  P.grads = o; o = al(o + 4 * (size_t)P.nparam);
  P.m1 = o; o = al(o + 4 * (size_t)P.nparam);
  P.m2 = o; o = al(o + 4 * (size_t)P.nparam);
  P.wcopies = o;
  for (int k = 0; k < NCONV; ++k) {
    Conv& c = P.cv[k];
    c.wf = o; o = al(o + 2 * 9 * (size_t)c.Ck * c.co);
    c.wb = o; o = al(o + 2 * 9 * (size_t)c.Ck * c.co);
  }
  P.loss = o; o = al(o + 8);
  P.act = o;
  const size_t B = d.max_batch;
  const int cw[4] = {c0, c1, c2, c3};
  auto take = [&](size_t elems) { size_t r = o; o = al(o + 2 * elems * B); return r; };
  P.xin = take(16 * (size_t)npix_lvl(d, 0));
  for (int l = 0; l < 4; ++l) {
    P.e_a[l] = take((size_t)cw[l] * npix_lvl(d, l));
    P.e_b[l] = take((size_t)cw[l] * npix_lvl(d, l));
  }
  for (int l = 0; l < 3; ++l) {
    P.pool[l] = take((size_t)cw[l] * npix_lvl(d, l + 1));
    P.cat[l] = take((size_t)(cw[l + 1] + cw[l]) * npix_lvl(d, l));
    P.d_a[l] = take((size_t)cw[l] * npix_lvl(d, l));
    P.d_b[l] = take((size_t)cw[l] * npix_lvl(d, l));
    P.gcat[l] = take((size_t)(cw[l + 1] + cw[l]) * npix_lvl(d, l));
    P.gskip[l] = take((size_t)cw[l] * npix_lvl(d, l));
  }
  for (int l = 0; l < 4; ++l) {
    // two gradient scratch tensors per level, wide enough for its channels
    // and for the pooled gradient of the level above
    const size_t cmax = std::max(cw[l], l > 0 ? cw[l - 1] : 0);
    P.gbig1[l] = take(cmax * npix_lvl(d, l));
    P.gbig2[l] = take(cmax * npix_lvl(d, l));
  }
  P.y = o; o = al(o + 4 * B * d.c_out * (size_t)npix_lvl(d, 0));
  P.gy = o; o = al(o + 4 * B * d.c_out * (size_t)npix_lvl(d, 0));
  // per-chunk partial sums of the parameter gradients (one reduction at a
  // time on the stream, so one buffer serves all), for every batch size up to
  // max_batch; and the per-workgroup squared errors of the loss
  size_t part = 0;
  for (int b = 1; b <= d.max_batch; ++b) {
    for (int k = 0; k < NCONV; ++k) {
      const Conv& c = P.cv[k];
      const int l = conv_level(k);
      const WgShape S = wgrad_shape(c.Ck, c.co, b, d.H >> l, d.W >> l);
      part = std::max(part, (size_t)S.gx * (9 * c.ci * c.co + c.co));
    }
    part = std::max(part, (size_t)head_chunks((long long)b * npix_lvl(d, 0), c0) *
                              ((size_t)c0 * d.c_out + d.c_out));
  }
  P.part = o; o = al(o + 4 * part);
  P.loss_part = o; o = al(o + 8 * (size_t)blocks(B * npix_lvl(d, 0)));
  P.total = o;
  return true;
}

lbaxi_status validate(const lbnn_desc* d) {
  if (!d) return nfail(LBAXI_EINVAL, "NULL desc");
  if (d->H < 8 || d->W < 8 || d->H % 8 || d->W % 8) return nfail(LBAXI_EINVAL, "H, W must be multiples of 8");
  if (d->c_in < 1 || d->c_in > 16) return nfail(LBAXI_EINVAL, "c_in must be in 1..16");
  if (d->c_out < 1 || d->c_out > 8) return nfail(LBAXI_EINVAL, "c_out must be in 1..8");
  for (int k = 0; k < 4; ++k)
    if (d->widths[k] < 32 || d->widths[k] > 256 || d->widths[k] % 32)
      return nfail(LBAXI_EINVAL, "widths must be multiples of 32 in 32..256");
  if (d->max_batch < 1) return nfail(LBAXI_EINVAL, "max_batch must be >= 1");
  // every tensor stays below 2^31 elements / 8-channel vectors (32-bit indexing)
  if ((long long)d->max_batch * d->H * d->W * 512 >= (1LL << 31))
    return nfail(LBAXI_EINVAL, "max_batch * H * W must be below 2^22");
  return LBAXI_OK;
}

}  // namespace

struct lbnn_s {
  Plan P;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int batch = 0;       // batch of the last forward
  long long step = 0;  // Adam step counter
  bool wdirty = true;  // BF16 copies out of date
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float* params() const { return at<float>(P.params); }
  float* grads() const { return at<float>(P.grads); }
  bf16s* act(size_t off) const { return at<bf16s>(off); }
};

namespace {

lbaxi_status refresh_weights(lbnn_t* h) {
  if (!h->wdirty) return LBAXI_OK;
  for (int k = 0; k < NCONV; ++k) {
    const Conv& c = h->P.cv[k];
    hipLaunchKernelGGL(k_cast_w, dim3(blocks(9LL * c.Ck * c.co)), dim3(256), 0, h->stream,
                       h->params() + c.off_W, h->at<bf16s>(c.wf), h->at<bf16s>(c.wb), c.ci, c.Ck,
                       c.co);
  }
  NCHK(hipGetLastError());
  h->wdirty = false;
  return LBAXI_OK;
}

lbaxi_status conv(lbnn_t* h, const Conv& c, const bf16s* in, bf16s* out, int lvl, int B,
                  bool adjoint, const bf16s* mask) {
  ConvArgs A;
  A.B = B;
  A.H = h->P.d.H >> lvl;
  A.W = h->P.d.W >> lvl;
  A.in = in;
  A.out = out;
  A.mask = mask;
  if (!adjoint) {
    A.wt = h->at<bf16s>(c.wf);
    A.bias = h->params() + c.off_b;
    A.Ck = c.Ck;
    A.Cn = c.co;
    A.sign = 1;
    A.act = 1;
  } else {
    A.wt = h->at<bf16s>(c.wb);
    A.bias = nullptr;
    A.Ck = c.co;
    A.Cn = c.Ck;
    A.sign = -1;
    A.act = 0;
  }
  const long long npix = (long long)B * A.H * A.W;
  // 2 x 2 blocks per wave where the output width allows, else 4 x 1
  // Image rows wide enough for a row segment: the halo variant (every input
  // row read once per stage rather than once per tap).
  {
    void* rf = nullptr;
    int tw = 0, nt = 0;
    if (A.W % 128 == 0 && A.Cn % 64 == 0) {
      rf = (void*)&k_conv_row<128, 64>; tw = 128; nt = 64;
    } else if (A.W % 128 == 0 && A.Cn % 32 == 0) {
      rf = (void*)&k_conv_row<128, 32>; tw = 128; nt = 32;
    } else if (A.W % 64 == 0 && A.Cn % 64 == 0) {
      rf = (void*)&k_conv_row<64, 64>; tw = 64; nt = 64;
    } else if (A.W % 32 == 0 && A.Cn % 128 == 0) {
      rf = (void*)&k_conv_row<32, 128>; tw = 32; nt = 128;
    }
    if (rf) {
      dim3 grid((unsigned)((long long)B * A.H * (A.W / tw)), A.Cn / nt);
      void* args[] = {&A};
      NCHK(hipLaunchKernel(rf, grid, dim3(256), args, 0, h->stream));
      return LBAXI_OK;
    }
  }
  // otherwise a flat pixel tile, largest first, down to 64 x 64 while the
  // grid would leave CUs idle
  int PT, NT;
  void* fn;
  auto wgs = [&](int pt, int nt) { return (long long)blocks(npix, pt) * (A.Cn / nt); };
  if (A.Cn % 128 == 0 && wgs(128, 128) >= 1024) {
    PT = 128; NT = 128; fn = (void*)&k_conv<128, 128, 2, 2>;
  } else if (A.Cn % 64 == 0 && wgs(128, 64) >= 1024) {
    PT = 128; NT = 64; fn = (void*)&k_conv<128, 64, 2, 1>;
  } else if (A.Cn % 64 == 0) {
    PT = 64; NT = 64; fn = (void*)&k_conv<64, 64, 1, 1>;
  } else {
    PT = 256; NT = 32; fn = (void*)&k_conv<256, 32, 2, 1>;
  }
  dim3 grid(blocks(npix, PT), A.Cn / NT);
  void* args[] = {&A};
  NCHK(hipLaunchKernel(fn, grid, dim3(256), args, 0, h->stream));
  return LBAXI_OK;
}

// Sum of the per-chunk partials part[nchunk][n] into out[n] (fixed order).
// Runs per element: doubled while each run keeps at least 8 chunks and the
// grid stays under 1024 workgroups, at most 16.
lbaxi_status sum_chunks(lbnn_t* h, float* out, long long n, long long nchunk) {
  int G = 1;
  while (G < 16 && nchunk / (2 * G) >= 8 && blocks(n, 256 / G) < 1024) G *= 2;
  void* fn = G == 16 ? (void*)&k_sum_chunks<16>
             : G == 8 ? (void*)&k_sum_chunks<8>
             : G == 4 ? (void*)&k_sum_chunks<4>
             : G == 2 ? (void*)&k_sum_chunks<2>
                      : (void*)&k_sum_chunks<1>;
  const float* part = h->at<float>(h->P.part);
  int nc = (int)nchunk;
  void* args[] = {&part, &out, &n, &nc};
  NCHK(hipLaunchKernel(fn, dim3((unsigned)blocks(n, 256 / G)), dim3(256), args, 0, h->stream));
  return LBAXI_OK;
}

lbaxi_status wgrad(lbnn_t* h, const Conv& c, const bf16s* x, const bf16s* gz, int lvl, int B) {
  WgradArgs A;
  A.x = x;
  A.gz = gz;
  A.part = h->at<float>(h->P.part);
  A.B = B;
  A.H = h->P.d.H >> lvl;
  A.W = h->P.d.W >> lvl;
  A.Cx = c.Ck;
  A.Ci = c.ci;
  A.Co = c.co;
  const long long npix = (long long)B * A.H * A.W;
  const WgShape S = wgrad_shape(c.Ck, c.co, B, A.H, A.W);
  A.cib = S.cib;
  A.cob = S.cob;
  A.chunk = S.chunk;
  dim3 grid((unsigned)S.gx, (unsigned)S.gy);
  void* fn;
  if (S.row) {
    // narrow outputs on wide rows: row segments, every input row staged once
    // for all nine taps
    fn = (void*)&k_wgrad_row;
  } else {
    fn = S.MB == 2 ? (S.NB == 2 ? (void*)&k_wgrad<2, 2> : (void*)&k_wgrad<2, 1>)
                   : (S.NB == 2 ? (void*)&k_wgrad<1, 2> : (void*)&k_wgrad<1, 1>);
  }
  void* args[] = {&A};
  NCHK(hipLaunchKernel(fn, grid, dim3(256), args, 0, h->stream));
  // dW then db: contiguous in the parameter vector as in each chunk's slice
  return sum_chunks(h, h->grads() + c.off_W, 9LL * c.ci * c.co + c.co, S.gx);
}

}  // namespace

extern "C" {

lbaxi_status lbnn_workspace_bytes(const lbnn_desc* d, size_t* bytes) {
  lbaxi_status s = validate(d);
  if (s != LBAXI_OK) return s;
  if (!bytes) return nfail(LBAXI_EINVAL, "NULL bytes");
  Plan P;
  plan(*d, P);
  *bytes = P.total;
  return LBAXI_OK;
}

lbaxi_status lbnn_create(const lbnn_desc* d, void* d_workspace, size_t bytes, void* hip_stream,
                         lbnn_t** out) {
  if (!out) return nfail(LBAXI_EINVAL, "NULL out");
  *out = nullptr;
  size_t need;
  lbaxi_status s = lbnn_workspace_bytes(d, &need);
  if (s != LBAXI_OK) return s;
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return nfail(LBAXI_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < need) return nfail(LBAXI_ENOMEM, "workspace smaller than lbnn_workspace_bytes");
  lbnn_t* h = new (std::nothrow) lbnn_s();
  if (!h) return nfail(LBAXI_ENOMEM, "host allocation failed");
  plan(*d, h->P);
  h->ws = static_cast<char*>(d_workspace);
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  const long long n = h->P.nparam;
  for (size_t off : {h->P.params, h->P.grads, h->P.m1, h->P.m2})
    hipLaunchKernelGGL(k_zero, dim3(blocks(n)), dim3(256), 0, h->stream, h->at<float>(off), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    delete h;
    return nfail(LBAXI_EDEVICE, hipGetErrorString(e));
  }
  *out = h;
  return LBAXI_OK;
}

void lbnn_destroy(lbnn_t* h) { delete h; }

lbaxi_status lbnn_param_count(const lbnn_t* h, int64_t* n) {
  if (!h || !n) return nfail(LBAXI_EINVAL, "NULL argument");
  *n = h->P.nparam;
  return LBAXI_OK;
}

lbaxi_status lbnn_set_params(lbnn_t* h, const float* d_params) {
  if (!h || !d_params) return nfail(LBAXI_EINVAL, "NULL argument");
  NCHK(hipMemcpyAsync(h->params(), d_params, 4 * (size_t)h->P.nparam, hipMemcpyDeviceToDevice,
                      h->stream));
  const long long n = h->P.nparam;
  for (size_t off : {h->P.m1, h->P.m2})
    hipLaunchKernelGGL(k_zero, dim3(blocks(n)), dim3(256), 0, h->stream, h->at<float>(off), n);
  NCHK(hipGetLastError());
  h->step = 0;
  h->wdirty = true;
  return LBAXI_OK;
}

lbaxi_status lbnn_get_params(lbnn_t* h, float* d_params) {
  if (!h || !d_params) return nfail(LBAXI_EINVAL, "NULL argument");
  NCHK(hipMemcpyAsync(d_params, h->params(), 4 * (size_t)h->P.nparam, hipMemcpyDeviceToDevice,
                      h->stream));
  return LBAXI_OK;
}

lbaxi_status lbnn_forward(lbnn_t* h, const float* d_x, float* d_y, int32_t B) {
  if (!h || !d_x) return nfail(LBAXI_EINVAL, "NULL argument");
  const Plan& P = h->P;
  if (B < 1 || B > P.d.max_batch) return nfail(LBAXI_EINVAL, "batch out of range");
  lbaxi_status s;
  if ((s = refresh_weights(h)) != LBAXI_OK) return s;
  const int c0 = P.d.widths[0], c1 = P.d.widths[1], c2 = P.d.widths[2], c3 = P.d.widths[3];
  const int cw[4] = {c0, c1, c2, c3};
  const long long np0 = (long long)B * npix_lvl(P.d, 0);
  hipLaunchKernelGGL(k_input, dim3(blocks(np0)), dim3(256), 0, h->stream, d_x,
                     h->act(P.xin), np0, P.d.c_in);
  NCHK(hipGetLastError());
  const bf16s* x = h->act(P.xin);
  for (int l = 0; l < 4; ++l) {
    if (l > 0) {
      const int Hh = P.d.H >> (l - 1), Ww = P.d.W >> (l - 1);
      hipLaunchKernelGGL(k_pool, dim3(blocks((long long)B * (Hh / 2) * (Ww / 2) * cw[l - 1] / 8)),
                         dim3(256), 0, h->stream, h->act(P.e_b[l - 1]), h->act(P.pool[l - 1]), B,
                         Hh, Ww, cw[l - 1]);
      NCHK(hipGetLastError());
      x = h->act(P.pool[l - 1]);
    }
    if ((s = conv(h, P.cv[2 * l], x, h->act(P.e_a[l]), l, B, false, nullptr)) != LBAXI_OK) return s;
    if ((s = conv(h, P.cv[2 * l + 1], h->act(P.e_a[l]), h->act(P.e_b[l]), l, B, false, nullptr)) !=
        LBAXI_OK)
      return s;
  }
  const bf16s* below = h->act(P.e_b[3]);
  for (int l = 2; l >= 0; --l) {
    const int Hl = P.d.H >> l, Wl = P.d.W >> l;
    const long long tot = (long long)B * Hl * Wl * (cw[l + 1] + cw[l]) / 8;
    hipLaunchKernelGGL(k_upcat, dim3(blocks(tot)), dim3(256), 0, h->stream, below,
                       h->act(P.e_b[l]), h->act(P.cat[l]), B, Hl, Wl, cw[l + 1], cw[l]);
    NCHK(hipGetLastError());
    const int ka = D2A + 2 * (2 - l);
    if ((s = conv(h, P.cv[ka], h->act(P.cat[l]), h->act(P.d_a[l]), l, B, false, nullptr)) != LBAXI_OK)
      return s;
    if ((s = conv(h, P.cv[ka + 1], h->act(P.d_a[l]), h->act(P.d_b[l]), l, B, false, nullptr)) !=
        LBAXI_OK)
      return s;
    below = h->act(P.d_b[l]);
  }
  float* y = d_y ? d_y : h->at<float>(P.y);
  hipLaunchKernelGGL(k_head, dim3(blocks(np0)), dim3(256), 0, h->stream, h->act(P.d_b[0]),
                     h->params() + P.off_hW, h->params() + P.off_hb, h->at<float>(P.y),
                     (const float*)nullptr, (float*)nullptr, (double*)nullptr, np0, c0, P.d.c_out,
                     0.0);
  NCHK(hipGetLastError());
  if (d_y)
    NCHK(hipMemcpyAsync(y, h->at<float>(P.y), 4 * (size_t)np0 * P.d.c_out,
                        hipMemcpyDeviceToDevice, h->stream));
  h->batch = B;
  return LBAXI_OK;
}

lbaxi_status lbnn_backward(lbnn_t* h, const float* d_target, float* d_grads, double* host_loss) {
  if (!h || !d_target) return nfail(LBAXI_EINVAL, "NULL argument");
  if (h->batch < 1) return nfail(LBAXI_ESTATE, "no forward pass to differentiate");
  const Plan& P = h->P;
  const int B = h->batch;
  const int c0 = P.d.widths[0], c1 = P.d.widths[1], c2 = P.d.widths[2], c3 = P.d.widths[3];
  const int cw[4] = {c0, c1, c2, c3};
  const long long np0 = (long long)B * npix_lvl(P.d, 0);
  lbaxi_status s;
  // every parameter gradient and the loss are written (not accumulated) below
  // head: y again with the target, then its backward into gz of d0b
  hipLaunchKernelGGL(k_head, dim3(blocks(np0)), dim3(256), 0, h->stream, h->act(P.d_b[0]),
                     h->params() + P.off_hW, h->params() + P.off_hb, h->at<float>(P.y), d_target,
                     h->at<float>(P.gy), h->at<double>(P.loss_part), np0, c0, P.d.c_out,
                     1.0 / ((double)np0 * P.d.c_out));
  hipLaunchKernelGGL(k_sum_chunks_d, dim3(1), dim3(256), 0, h->stream,
                     h->at<double>(P.loss_part), h->at<double>(P.loss), (int)blocks(np0));
  hipLaunchKernelGGL(k_head_back, dim3(blocks(np0)), dim3(256), 0, h->stream, h->act(P.d_b[0]),
                     h->at<float>(P.gy), h->params() + P.off_hW, h->act(P.gbig1[0]), np0, c0,
                     P.d.c_out);
  const long long nh = head_chunks(np0, c0);
  hipLaunchKernelGGL(k_head_wgrad, dim3((unsigned)nh), dim3(256), 0, h->stream, h->act(P.d_b[0]),
                     h->at<float>(P.gy), h->at<float>(P.part), np0, c0, P.d.c_out);
  NCHK(hipGetLastError());
  // head.W and head.b are contiguous in the parameter vector, as in a chunk
  if ((s = sum_chunks(h, h->grads() + P.off_hW, (long long)c0 * P.d.c_out + P.d.c_out, nh)) !=
      LBAXI_OK)
    return s;
  // decoder levels 0, 1, 2: gz of the block output is in gbig1[l]
  for (int l = 0; l <= 2; ++l) {
    const int ka = D2A + 2 * (2 - l);
    const Conv& ca = P.cv[ka];
    const Conv& cb = P.cv[ka + 1];
    bf16s* gzb = h->act(P.gbig1[l]);
    bf16s* gza = h->act(P.gbig2[l]);
    if ((s = wgrad(h, cb, h->act(P.d_a[l]), gzb, l, B)) != LBAXI_OK) return s;
    if ((s = conv(h, cb, gzb, gza, l, B, true, h->act(P.d_a[l]))) != LBAXI_OK) return s;
    if ((s = wgrad(h, ca, h->act(P.cat[l]), gza, l, B)) != LBAXI_OK) return s;
    if ((s = conv(h, ca, gza, h->act(P.gcat[l]), l, B, true, nullptr)) != LBAXI_OK) return s;
    // split: upsampled part -> gz of the level below's block output (masked by
    // that activation's derivative), skip part -> gskip[l]
    const int Hl = P.d.H >> l, Wl = P.d.W >> l;
    const bf16s* u = l < 2 ? h->act(P.d_b[l + 1]) : h->act(P.e_b[3]);
    bf16s* gu = h->act(P.gbig1[l + 1]);
    const long long tot =
        ((long long)B * (Hl / 2) * (Wl / 2) * cw[l + 1] + (long long)B * Hl * Wl * cw[l]) / 8;
    hipLaunchKernelGGL(k_upcat_back, dim3(blocks(tot)), dim3(256), 0, h->stream,
                       h->act(P.gcat[l]), u, gu, h->act(P.gskip[l]), B, Hl, Wl, cw[l + 1], cw[l]);
    NCHK(hipGetLastError());
  }
  // encoder levels 3, 2, 1, 0: gz of e_b[l] in gbig1[l]
  for (int l = 3; l >= 0; --l) {
    const Conv& ca = P.cv[2 * l];
    const Conv& cb = P.cv[2 * l + 1];
    bf16s* gzb = h->act(P.gbig1[l]);
    bf16s* gza = h->act(P.gbig2[l]);
    if ((s = wgrad(h, cb, h->act(P.e_a[l]), gzb, l, B)) != LBAXI_OK) return s;
    if ((s = conv(h, cb, gzb, gza, l, B, true, h->act(P.e_a[l]))) != LBAXI_OK) return s;
    const bf16s* xin = l > 0 ? h->act(P.pool[l - 1]) : h->act(P.xin);
    if (l == 0) {
      // first layer: padded 16 input channels, gradient of the input unused
      if ((s = wgrad(h, ca, xin, gza, l, B)) != LBAXI_OK) return s;
      break;
    }
    if ((s = wgrad(h, ca, xin, gza, l, B)) != LBAXI_OK) return s;
    // gradient of the pooled input, then into e_b[l-1] with its skip part
    bf16s* gp = h->act(P.gbig1[l]);  // gzb is dead now
    if ((s = conv(h, ca, gza, gp, l, B, true, nullptr)) != LBAXI_OK) return s;
    const int Hh = P.d.H >> (l - 1), Ww = P.d.W >> (l - 1);
    hipLaunchKernelGGL(k_pool_back, dim3(blocks((long long)B * Hh * Ww * cw[l - 1] / 8)), dim3(256), 0,
                       h->stream, gp, h->act(P.gskip[l - 1]), h->act(P.e_b[l - 1]),
                       h->act(P.gbig1[l - 1]), B, Hh, Ww, cw[l - 1]);
    NCHK(hipGetLastError());
  }
  if (d_grads)
    NCHK(hipMemcpyAsync(d_grads, h->grads(), 4 * (size_t)P.nparam, hipMemcpyDeviceToDevice,
                        h->stream));
  if (host_loss) {
    double L;
    NCHK(hipMemcpyAsync(&L, h->at<double>(P.loss), 8, hipMemcpyDeviceToHost, h->stream));
    NCHK(hipStreamSynchronize(h->stream));
    *host_loss = L / ((double)np0 * P.d.c_out);
  }
  return LBAXI_OK;
}

lbaxi_status lbnn_adam(lbnn_t* h, float lr, float b1, float b2, float eps) {
  if (!h) return nfail(LBAXI_EINVAL, "NULL handle");
  h->step += 1;
  const float c1 = 1.0f - powf(b1, (float)h->step), c2 = 1.0f - powf(b2, (float)h->step);
  WCopies W;
  for (int q = 0; q < NCONV; ++q) {
    const Conv& c = h->P.cv[q];
    W.off[q] = c.off_W;
    W.ci[q] = c.ci;
    W.Ck[q] = c.Ck;
    W.co[q] = c.co;
    W.wf[q] = h->at<bf16s>(c.wf);
    W.wb[q] = h->at<bf16s>(c.wb);
  }
  hipLaunchKernelGGL(k_adam, dim3(blocks(h->P.nparam)), dim3(256), 0, h->stream, h->params(),
                     h->grads(), h->at<float>(h->P.m1), h->at<float>(h->P.m2), h->P.nparam, lr, b1,
                     b2, eps, c1, c2, W);
  NCHK(hipGetLastError());
  // copies that were current stay current (the step wrote them); copies out
  // of date (parameters set since the last cast) are cast before next use
  return LBAXI_OK;
}

lbaxi_status lbnn_train_step(lbnn_t* h, const float* d_x, const float* d_target, int32_t batch,
                             float lr, double* host_loss) {
  lbaxi_status s = lbnn_forward(h, d_x, nullptr, batch);
  if (s == LBAXI_OK) s = lbnn_backward(h, d_target, nullptr, host_loss);
  if (s == LBAXI_OK) s = lbnn_adam(h, lr, 0.9f, 0.999f, 1e-8f);
  return s;
}

lbaxi_status lbnn_to_fields(lbnn_t* h, const float* d_y, int32_t batch, const float* sc,
                            const float* of, int32_t smooth, float* const* d_fields) {
  if (!h || !d_y || !sc || !of || !d_fields) return nfail(LBAXI_EINVAL, "NULL argument");
  if (batch < 1 || batch > h->P.d.max_batch) return nfail(LBAXI_EINVAL, "batch out of range");
  if (smooth != 0 && smooth != 1) return nfail(LBAXI_EINVAL, "smooth must be 0 or 1");
  FieldOut o;
  for (int k = 0; k < 8; ++k) {
    const bool use = k < h->P.d.c_out;
    o.p[k] = use ? d_fields[k] : nullptr;
    o.sc[k] = use ? sc[k] : 0.0f;
    o.of[k] = use ? of[k] : 0.0f;
  }
  const long long np = (long long)batch * npix_lvl(h->P.d, 0);
  hipLaunchKernelGGL(k_to_fields, dim3(blocks(np)), dim3(256), 0, h->stream, d_y, (int)batch,
                     h->P.d.H, h->P.d.W, h->P.d.c_out, (int)smooth, o);
  NCHK(hipGetLastError());
  return LBAXI_OK;
}

lbaxi_status lbnn_mfma_selftest(int32_t* d_counter, void* hip_stream, int32_t* host_mismatches) {
  if (!host_mismatches || !d_counter) return nfail(LBAXI_EINVAL, "NULL argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, st, d_counter, 0);
  hipLaunchKernelGGL(k_mfma_selftest, dim3(1), dim3(64), 0, st, d_counter);
  NCHK(hipGetLastError());
  int bad = -1;
  NCHK(hipMemcpyAsync(&bad, d_counter, sizeof(int), hipMemcpyDeviceToHost, st));
  NCHK(hipStreamSynchronize(st));
  *host_mismatches = bad;
  return LBAXI_OK;
}

const char* lbnn_last_error(void) { return g_nerr.c_str(); }

}  // extern "C"
