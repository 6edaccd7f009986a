// ffs_surrogate: gfx950 kernels of the learned offspring pre-screen (the
// DeepSets surrogate declared in include/ffs_surrogate.h).
//
// Mapping onto CDNA4
//   * The only chromosome-dependent input is a job's rank, which takes n
//     values, so layers 1 and 2 run once per (job, rank) pair: a Q = n^2 row
//     table. Its products with W2 (forward) and the two backward products run
//     on the matrix cores: v_mfma_f32_32x32x16_bf16, 64 x 64 output tiles per
//     256-thread workgroup (2 x 2 waves of 32 x 32), K staged through LDS in
//     slices of 32. Layer-1 activations and the layer-2 output gradient are
//     built in the loaders straight into LDS as bf16, never stored.
//   * A batch's forward is a gather of table rows per chromosome; its
//     backward aggregates the output gradient per table row (the gradient of
//     every row of a chromosome is the same vector w3 * dy / n, masked), so
//     dW2 and dH1 are products over the Q table rows, not over batch x n.
//   * No float atomics: every sum runs in a fixed order (per-lane sequential,
//     fixed lane trees, per-block partials reduced in block order), so each
//     call repeats bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "ffs_surrogate.h"

namespace {

constexpr int H = FFS_SG_HIDDEN;
constexpr int kW1 = 0;                  // [4][H]
constexpr int kB1 = 4 * H;              // [H]
constexpr int kW2 = 5 * H;              // [H][H]
constexpr int kB2 = 5 * H + H * H;      // [H]
constexpr int kW3 = 6 * H + H * H;      // [H]
constexpr int kB3 = 7 * H + H * H;      // [1]
static_assert(kB3 + 1 == FFS_SG_PARAMS, "parameter layout");

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS row stride in bf16 elements
constexpr int kChunk = 256;                               // table rows per dW2 partial
constexpr int kRowChunk = 32;                             // table rows per db2 partial
constexpr int kBatchChunk = 64;                           // chromosomes per head partial
constexpr int kDChunk = 256;                              // chromosomes per D partial
constexpr int kHeaderBytes = 256;  // head of the training workspace: status word first, as ffs_status reads it

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// float32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ u32x4 pack8(const float *v) {
  u32x4 r;
#pragma unroll
  for (int j = 0; j < 4; ++j) r[j] = bf16_bits(v[2 * j]) | (bf16_bits(v[2 * j + 1]) << 16);
  return r;
}

// Layer 1 before the ReLU for job k at rank v / n: c_k + rank * W1[0], float32.
__device__ __forceinline__ float layer1(const float *ctab, const float *theta, int k, float rank,
                                        int h) {
  return __fadd_rn(ctab[k * H + h], __fmul_rn(rank, theta[kW1 + h]));
}

__device__ __forceinline__ float rank_of(int v, int n) { return __fdiv_rn((float)v, (float)n); }

// Layer-2 output gradient of table row q at unit o (before its bf16 rounding).
__device__ __forceinline__ float out_grad(const float *H2, const float *D, const float *theta, int q,
                                          int o, float fn) {
  return H2[(size_t)q * H + o] > 0.f ? __fdiv_rn(__fmul_rn(D[q], theta[kW3 + o]), fn) : 0.f;
}

struct TileLds {
  uint16_t a[BM * LDK];
  uint16_t b[BN * LDK];
};

// acc (this wave's 32 x 32 part of a 64 x 64 tile) += A[64 x K] B[K x 64].
// fa(r, k, v8) fills A[r][k..k+7] and fb(c, k, v8) fills B[k..k+7][c] as
// float32 values, rounded here to bf16; each thread fills one 8-wide slice of
// A and of B per K slice.
template <class FA, class FB>
__device__ __forceinline__ void mma_tile(int k_total, FA fa, FB fb, TileLds &s, f32x16 &acc) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
  const int r = t >> 2, kc = (t & 3) * 8;
  const int arow = (wm * 32 + (lane & 31)) * LDK, brow = (wn * 32 + (lane & 31)) * LDK;
  const int koff = 8 * (lane >> 5);
  for (int k0 = 0; k0 < k_total; k0 += BK) {
    float va[8], vb[8];
    fa(r, k0 + kc, va);
    fb(r, k0 + kc, vb);
    *(u32x4 *)&s.a[r * LDK + kc] = pack8(va);
    *(u32x4 *)&s.b[r * LDK + kc] = pack8(vb);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      const u32x4 av = *(const u32x4 *)&s.a[arow + kk + koff];
      const u32x4 bv = *(const u32x4 *)&s.b[brow + kk + koff];
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av),
                                                    __builtin_bit_cast(bf16x8, bv), acc, 0, 0, 0);
    }
    __syncthreads();
  }
}

// Tile coordinates of accumulator element e of this lane.
__device__ __forceinline__ int acc_row(int e) {
  const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1;
  return wm * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
}
__device__ __forceinline__ int acc_col() {
  const int lane = threadIdx.x & 63, wn = (threadIdx.x >> 6) & 1;
  return wn * 32 + (lane & 31);
}

// ---------------------------------------------------------------------------
// Features, layer-1 constants, bf16 copies.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void features_kernel(ffs_instance in, float *feats) {
  __shared__ int32_t smax[256];
  const int n = in.n_active, g = in.n_stages, om = in.o_max;
  int32_t my_max = 0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int j = in.active[k];
    int32_t tot = 0;
    for (int s = in.first_stage[j]; s < g; ++s) {
      const int32_t *row = in.proc + ((size_t)j * g + s) * om;
      int32_t best = row[0];
      for (int m = 1; m < in.n_machines[s]; ++m) best = row[m] < best ? row[m] : best;
      tot += best;
    }
    my_max = tot > my_max ? tot : my_max;
  }
  smax[threadIdx.x] = my_max;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h && smax[threadIdx.x + h] > smax[threadIdx.x])
      smax[threadIdx.x] = smax[threadIdx.x + h];
    __syncthreads();
  }
  const float scale = (float)(smax[0] > 1 ? smax[0] : 1);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int j = in.active[k];
    int64_t tot = 0;
    for (int s = in.first_stage[j]; s < g; ++s) {
      const int32_t *row = in.proc + ((size_t)j * g + s) * om;
      int32_t best = row[0];
      for (int m = 1; m < in.n_machines[s]; ++m) best = row[m] < best ? row[m] : best;
      tot += best;
    }
    const int64_t ready = in.ready[j];
    const int64_t start = ready > in.rs ? ready : in.rs;
    const int64_t slack = (int64_t)in.due[j] - start - tot;
    const int64_t rel = ready - in.rs > 0 ? ready - in.rs : 0;
    feats[4 * k + 0] = __fdiv_rn((float)tot, scale);
    feats[4 * k + 1] = __fdiv_rn((float)slack, scale);
    feats[4 * k + 2] = __fdiv_rn((float)rel, scale);
    feats[4 * k + 3] = 0.f;
  }
}

// c_k = ((b1 + f0 W1[1]) + f1 W1[2]) + f2 W1[3], float32 in this order.
__global__ __launch_bounds__(256) void ctab_kernel(const float *theta, const float *feats, int n,
                                                   float *ctab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * H) return;
  const int k = i / H, h = i % H;
  float c = __fadd_rn(theta[kB1 + h], __fmul_rn(feats[4 * k + 0], theta[kW1 + H + h]));
  c = __fadd_rn(c, __fmul_rn(feats[4 * k + 1], theta[kW1 + 2 * H + h]));
  c = __fadd_rn(c, __fmul_rn(feats[4 * k + 2], theta[kW1 + 3 * H + h]));
  ctab[i] = c;
}

__global__ __launch_bounds__(256) void refresh_kernel(const float *theta, uint16_t *w2b,
                                                      uint16_t *w2tb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * H) return;
  const uint16_t b = (uint16_t)bf16_bits(theta[kW2 + i]);
  w2b[i] = b;
  w2tb[(i % H) * H + i / H] = b;
}

// ---------------------------------------------------------------------------
// Table forward: a2 = h1 . bf16(W2) + b2 for the Q = n^2 (job, rank) rows.
// SCORE: per-row dot products with w3 (4 column-block partials per row).
// TRAIN: h2 = max(a2, 0) stored, float32 [Q][H].
// grid (ceil(Q / 64), H / 64), 256 threads.
// ---------------------------------------------------------------------------
template <bool TRAIN>
__global__ __launch_bounds__(256) void table_fwd_kernel(const float *theta, const float *ctab,
                                                        const uint16_t *w2tb, int n, float *h2_out,
                                                        float *r_part) {
  __shared__ __align__(16) TileLds s;
  __shared__ float red[2][2][32];
  const int Q = n * n, m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  auto fa = [&](int r, int k, float *v) {
    const int q = m0 + r;
    if (q >= Q) {
      for (int j = 0; j < 8; ++j) v[j] = 0.f;
      return;
    }
    const int kj = q / n;
    const float rank = rank_of(q % n + 1, n);
    for (int j = 0; j < 8; ++j) v[j] = fmaxf(layer1(ctab, theta, kj, rank, k + j), 0.f);
  };
  auto fb = [&](int c, int k, float *v) {   // B[h][o] = W2[h][o], from the transpose
    const uint16_t *src = w2tb + (size_t)(n0 + c) * H + k;
    for (int j = 0; j < 8; ++j) v[j] = __uint_as_float((uint32_t)src[j] << 16);
  };
  f32x16 acc = {};
  mma_tile(H, fa, fb, s, acc);
  const int col = n0 + acc_col();
  const float b2 = theta[kB2 + col], w3 = theta[kW3 + col];
  const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1, wn = (threadIdx.x >> 6) & 1;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int q = m0 + acc_row(e);
    const float h2 = fmaxf(__fadd_rn(acc[e], b2), 0.f);
    if (TRAIN) {
      if (q < Q) h2_out[(size_t)q * H + col] = h2;
    } else {
      float p = __fmul_rn(w3, h2);
      // sum over the 32 columns of this wave (lanes with the same lane >> 5)
      for (int off = 1; off < 32; off <<= 1) p += __shfl_xor(p, off);
      if ((lane & 31) == 0) red[wm][wn][8 * (e >> 2) + 4 * (lane >> 5) + (e & 3)] = p;
    }
  }
  if (!TRAIN) {
    __syncthreads();
    const int t = threadIdx.x;
    if (t < BM) {
      const int q = m0 + t;
      if (q < Q) r_part[(size_t)blockIdx.y * Q + q] = red[t >> 5][0][t & 31] + red[t >> 5][1][t & 31];
    }
  }
}

__global__ __launch_bounds__(256) void table_sum_kernel(const float *r_part, int Q, float *table) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  float s = r_part[q];
  for (int b = 1; b < H / BN; ++b) s += r_part[(size_t)b * Q + q];
  table[q] = s;
}

// ---------------------------------------------------------------------------
// Training-step input check: every gene in 1..n and every target finite, else
// bit 0 of the status word; the later kernels of the step then do nothing.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1) void clear_status_kernel(int32_t *status) { status[0] = 0; }

__global__ __launch_bounds__(256) void validate_kernel(const int32_t *prio, const float *target,
                                                       int n, int B, int32_t *status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  bool bad = !(fabsf(target[b]) <= 3.0e38f);   // NaN or infinite
  for (int k = 0; k < n; ++k) {
    const int v = prio[(size_t)b * n + k];
    bad |= v < 1 || v > n;
  }
  if (bad) atomicOr(status, 1);
}

// ---------------------------------------------------------------------------
// Training targets: ln obj standardised within each group of `group`
// consecutive chromosomes (one population), mean and population standard
// deviation in float64; a constant group gets 0. One block of 256 threads per
// group: thread t sums its run of consecutive entries [g0 + t*c, g0 + (t+1)*c)
// in index order, c = ceil(group / 256), and the 256 partial sums are added by
// a fixed pairwise tree, so every run gives the same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_fixed(double v, double *buf) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) buf[t] += buf[t + w];
    __syncthreads();
  }
  const double out = buf[0];
  __syncthreads();
  return out;
}

__global__ __launch_bounds__(256) void targets_kernel(const int64_t *obj, int count, int group,
                                                     float *target, int32_t *status) {
  __shared__ double buf[256];
  const int g0 = blockIdx.x * group;
  const int g1 = g0 + group < count ? g0 + group : count;
  const int c = (g1 - g0 + 255) / 256;
  const int a = min(g0 + (int)threadIdx.x * c, g1), b = min(a + c, g1);
  double s = 0.0;
  bool bad = false;
  for (int i = a; i < b; ++i) {
    bad |= obj[i] <= 0;
    s += log((double)(obj[i] > 0 ? obj[i] : 1));
  }
  if (bad) atomicOr(status, 1);
  const double mean = block_sum_fixed(s, buf) / (double)(g1 - g0);
  double v = 0.0;
  for (int i = a; i < b; ++i) {
    const double d = log((double)(obj[i] > 0 ? obj[i] : 1)) - mean;
    v += d * d;
  }
  const double sd = sqrt(block_sum_fixed(v, buf) / (double)(g1 - g0));
  for (int i = g0 + threadIdx.x; i < g1; i += blockDim.x) {
    const double d = log((double)(obj[i] > 0 ? obj[i] : 1)) - mean;
    target[i] = sd > 0.0 ? (float)(d / sd) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Batch forward (pool order): z_b = (sum over k of h2[k][prio_bk]) / n,
// y_b = b3 + z_b . w3, dy_b = 2 (y_b - t_b) / B.
// One wave per chromosome, 4 units per lane.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void batch_fwd_kernel(const float *theta, const float *h2,
                                                       const int32_t *prio, const float *target,
                                                       int n, int B, float *z, float *dy,
                                                       float *sq, const int32_t *status) {
  if (status[0]) return;
  const int b = blockIdx.x, lane = threadIdx.x;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < n; ++k) {
    const int q = k * n + prio[(size_t)b * n + k] - 1;
    const float *row = h2 + (size_t)q * H;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += row[lane + 64 * j];
  }
  float part = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float zv = __fdiv_rn(acc[j], (float)n);
    z[(size_t)b * H + lane + 64 * j] = zv;
    part += __fmul_rn(theta[kW3 + lane + 64 * j], zv);
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  part = __shfl(part, 0);
  if (lane == 0) {
    const float y = __fadd_rn(theta[kB3], part);
    const float t = target[b];
    const float d = __fsub_rn(y, t);
    dy[b] = __fdiv_rn(__fmul_rn(2.f, d), (float)B);
    sq[b] = __fmul_rn(d, d);
  }
}

// Partials of D[k][v-1] = sum of dy_b over the chromosomes whose gene k is v:
// block (k, c) sums chromosomes [c * kDChunk, (c + 1) * kDChunk) in b order into
// part[c][k * n + v - 1]; the chunks are then added in chunk order.
__global__ __launch_bounds__(256) void dtable_kernel(const int32_t *prio, const float *dy, int n,
                                                     int B, float *part, const int32_t *status) {
  if (status[0]) return;
  __shared__ int32_t vals[kDChunk];
  __shared__ float dys[kDChunk];
  const int k = blockIdx.x, c = blockIdx.y;
  const int b0 = c * kDChunk, nb = B - b0 < kDChunk ? B - b0 : kDChunk;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    vals[i] = prio[(size_t)(b0 + i) * n + k];
    dys[i] = dy[b0 + i];
  }
  __syncthreads();
  for (int v = threadIdx.x + 1; v <= n; v += blockDim.x) {
    float s = 0.f;
    for (int i = 0; i < nb; ++i)
      if (vals[i] == v) s += dys[i];
    part[(size_t)c * n * n + k * n + v - 1] = s;
  }
}

// Partials of dw3, db3 and the loss over chromosomes [c * kBatchChunk, ...),
// b in order: part[c][0..H) = dw3, part[c][H] = db3, part[c][H + 1] = sum of squares.
__global__ __launch_bounds__(256) void head_kernel(const float *dy, const float *z, const float *sq,
                                                   int B, float *part, const int32_t *status) {
  if (status[0]) return;
  const int o = threadIdx.x, c = blockIdx.x;
  const int b0 = c * kBatchChunk, b1 = b0 + kBatchChunk < B ? b0 + kBatchChunk : B;
  float s = 0.f;
  for (int b = b0; b < b1; ++b) s += __fmul_rn(dy[b], z[(size_t)b * H + o]);
  float *out = part + (size_t)c * (H + 2);
  out[o] = s;
  if (o == 0) {
    float d = 0.f, l = 0.f;
    for (int b = b0; b < b1; ++b) {
      d += dy[b];
      l += sq[b];
    }
    out[H] = d;
    out[H + 1] = l;
  }
}

// The head partials added in chunk order: dw3, db3 and the loss (mean of squares).
__global__ __launch_bounds__(256) void head_sum_kernel(const float *part, int n_parts, int B,
                                                       float *grad, float *loss,
                                                       const int32_t *status) {
  if (status[0]) return;
  const int o = threadIdx.x;
  float s = 0.f;
  for (int c = 0; c < n_parts; ++c) s += part[(size_t)c * (H + 2) + o];
  grad[kW3 + o] = s;
  if (o == 0) {
    float d = 0.f, l = 0.f;
    for (int c = 0; c < n_parts; ++c) {
      d += part[(size_t)c * (H + 2) + H];
      l += part[(size_t)c * (H + 2) + H + 1];
    }
    grad[kB3] = d;
    loss[0] = __fdiv_rn(l, (float)B);
  }
}

// db2 partials: part[c][o] = sum of the layer-2 output gradient over rows of chunk c.
__global__ __launch_bounds__(256) void db2_part_kernel(const float *theta, const float *h2,
                                                       const float *D, int n, float *part,
                                                       const int32_t *status) {
  if (status[0]) return;
  const int Q = n * n, c = blockIdx.x, o = threadIdx.x;
  const int q1 = (c + 1) * kRowChunk < Q ? (c + 1) * kRowChunk : Q;
  float s = 0.f;
  for (int q = c * kRowChunk; q < q1; ++q) s += out_grad(h2, D, theta, q, o, (float)n);
  part[(size_t)c * H + o] = s;
}

// dH1 = bf16(G) . bf16(W2)^T over the table rows, masked by a1 > 0, reduced
// straight into per-block partials of dW1 (4 rows) and db1:
// part[blockIdx.x][f][h], f = 0 rank, 1..3 features, 4 bias.
// grid (ceil(Q / 64), H / 64), 256 threads.
__global__ __launch_bounds__(256) void bwd_h1_kernel(const float *theta, const float *ctab,
                                                     const float *feats, const float *h2,
                                                     const float *D, const uint16_t *w2b, int n,
                                                     float *part, const int32_t *status) {
  if (status[0]) return;
  __shared__ __align__(16) TileLds s;
  __shared__ float red[2][5][64];
  const int Q = n * n, m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const float fn = (float)n;
  auto fa = [&](int r, int k, float *v) {   // A[q][o] = G[q][o]
    const int q = m0 + r;
    for (int j = 0; j < 8; ++j) v[j] = q < Q ? out_grad(h2, D, theta, q, k + j, fn) : 0.f;
  };
  auto fb = [&](int c, int k, float *v) {   // B[o][h] = W2[h][o]
    const uint16_t *src = w2b + (size_t)(n0 + c) * H + k;
    for (int j = 0; j < 8; ++j) v[j] = __uint_as_float((uint32_t)src[j] << 16);
  };
  f32x16 acc = {};
  mma_tile(H, fa, fb, s, acc);
  const int h = n0 + acc_col();
  const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1;
  float p[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int q = m0 + acc_row(e);
    if (q >= Q) continue;
    const int kj = q / n;
    const float rank = rank_of(q % n + 1, n);
    const float d = layer1(ctab, theta, kj, rank, h) > 0.f ? acc[e] : 0.f;
    p[0] += __fmul_rn(rank, d);
    p[1] += __fmul_rn(feats[4 * kj + 0], d);
    p[2] += __fmul_rn(feats[4 * kj + 1], d);
    p[3] += __fmul_rn(feats[4 * kj + 2], d);
    p[4] += d;
  }
#pragma unroll
  for (int f = 0; f < 5; ++f) p[f] += __shfl_xor(p[f], 32);   // the two row halves of the wave
  if (lane < 32)
    for (int f = 0; f < 5; ++f) red[wm][f][acc_col()] = p[f];
  __syncthreads();
  const int t = threadIdx.x;
  for (int i = t; i < 5 * BN; i += blockDim.x) {
    const int f = i / BN, c = i % BN;
    part[((size_t)blockIdx.x * 5 + f) * H + n0 + c] = red[0][f][c] + red[1][f][c];
  }
}

// dW2 partials over one chunk of table rows: part[chunk][h][o] = sum over q of
// bf16(h1[q][h]) bf16(G[q][o]). grid (H / 64, H / 64, chunks), 256 threads.
__global__ __launch_bounds__(256) void bwd_w2_kernel(const float *theta, const float *ctab,
                                                     const float *h2, const float *D, int n,
                                                     float *part, const int32_t *status) {
  if (status[0]) return;
  __shared__ __align__(16) TileLds s;
  const int Q = n * n, m0 = blockIdx.x * BM, n0 = blockIdx.y * BN, qb = blockIdx.z * kChunk;
  const int qe = qb + kChunk < Q ? qb + kChunk : Q;
  const float fn = (float)n;
  auto fa = [&](int r, int k, float *v) {   // A[h][q] = h1[q][h]
    const int hh = m0 + r;
    for (int j = 0; j < 8; ++j) {
      const int q = qb + k + j;
      v[j] = q < qe ? fmaxf(layer1(ctab, theta, q / n, rank_of(q % n + 1, n), hh), 0.f) : 0.f;
    }
  };
  auto fb = [&](int c, int k, float *v) {   // B[q][o] = G[q][o]
    const int o = n0 + c;
    for (int j = 0; j < 8; ++j) {
      const int q = qb + k + j;
      v[j] = q < qe ? out_grad(h2, D, theta, q, o, fn) : 0.f;
    }
  };
  f32x16 acc = {};
  mma_tile(kChunk, fa, fb, s, acc);
  const int col = n0 + acc_col();
#pragma unroll
  for (int e = 0; e < 16; ++e)
    part[((size_t)blockIdx.z * H + m0 + acc_row(e)) * H + col] = acc[e];
}

// dst[i] = sum over p < n_parts of src[p * stride + i], p in order.
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float *src, int n_parts,
                                                           size_t stride, int count, float *dst,
                                                           const int32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count || status[0]) return;
  float s = src[i];
  for (int p = 1; p < n_parts; ++p) s += src[(size_t)p * stride + i];
  dst[i] = s;
}

// dW1 and db1 from the bwd_h1 partials: part[block][f][h] -> grad.
__global__ __launch_bounds__(256) void reduce_w1_kernel(const float *part, int n_blocks,
                                                        float *grad, const int32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;   // f * H + h
  if (i >= 5 * H || status[0]) return;
  float s = part[i];
  for (int p = 1; p < n_blocks; ++p) s += part[(size_t)p * 5 * H + i];
  if (i < 4 * H) grad[kW1 + i] = s;
  else grad[kB1 + i - 4 * H] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float *theta, float *m, float *v,
                                                   const float *grad, float lr, float c1, float c2,
                                                   uint16_t *w2b, uint16_t *w2tb,
                                                   const int32_t *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= FFS_SG_PARAMS || status[0]) return;
  const float g = grad[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  theta[i] = th;
  if (i >= kW2 && i < kW2 + H * H) {
    const int w = i - kW2;
    const uint16_t b = (uint16_t)bf16_bits(th);
    w2b[w] = b;
    w2tb[(w % H) * H + w / H] = b;
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
int grid1(int count) { return (count + 255) / 256; }

struct TableWs {
  float *ctab, *r_part;
  size_t total;
};

TableWs table_ws(void *ws, int n) {
  uint8_t *b = (uint8_t *)ws;
  TableWs L{};
  size_t off = 0;
  L.ctab = (float *)(b + off);
  off += align_up((size_t)n * H * 4, 256);
  L.r_part = (float *)(b + off);
  off += align_up((size_t)(H / BN) * n * n * 4, 256);
  L.total = off;
  return L;
}

struct TrainWs {
  int32_t *status;
  float *ctab, *h2, *D, *Dpart, *z, *dy, *sq, *head, *part1, *part_b2, *part_w2, *grad, *loss;
  size_t total;
};

TrainWs train_ws(void *ws, int n, int B) {
  uint8_t *b = (uint8_t *)ws;
  TrainWs L{};
  const size_t Q = (size_t)n * n, chunks = (Q + kChunk - 1) / kChunk, blocks = (Q + BM - 1) / BM;
  const size_t rchunks = (Q + kRowChunk - 1) / kRowChunk, dchunks = (B + kDChunk - 1) / kDChunk;
  const size_t hchunks = (B + kBatchChunk - 1) / kBatchChunk;
  size_t off = kHeaderBytes;
  L.status = (int32_t *)b;
  auto take = [&](size_t floats) {
    float *p = (float *)(b + off);
    off += align_up(floats * 4, 256);
    return p;
  };
  L.ctab = take((size_t)n * H);
  L.h2 = take(Q * H);
  L.D = take(Q);
  L.Dpart = take(dchunks * Q);
  L.z = take((size_t)B * H);
  L.dy = take(B);
  L.sq = take(B);
  L.head = take(hchunks * (H + 2));
  L.part1 = take(blocks * 5 * H);
  L.part_b2 = take(rchunks * H);
  L.part_w2 = take(chunks * H * H);
  L.grad = take(FFS_SG_PARAMS);
  L.loss = take(1);
  L.total = off;
  return L;
}

bool ok(hipError_t e) { return e == hipSuccess; }

}  // namespace

extern "C" {

int sg_refresh(ffs_surrogate *m, void *stream) {
  if (!m || !m->theta || !m->w2_bf16 || !m->w2t_bf16) return FFS_E_INVAL;
  hipLaunchKernelGGL(refresh_kernel, dim3(grid1(H * H)), dim3(256), 0, (hipStream_t)stream,
                     (const float *)m->theta, m->w2_bf16, m->w2t_bf16);
  return ok(hipGetLastError()) ? FFS_OK : FFS_E_DEVICE;
}

int sg_features(const ffs_instance *inst, float *feats, void *workspace, size_t workspace_bytes,
                void *stream) {
  (void)workspace;
  (void)workspace_bytes;
  if (!inst || !feats || inst->n_active < 1 || inst->n_active > FFS_SG_MAX_GENES ||
      inst->n_stages < 1 || inst->o_max < 1 || !inst->active || !inst->proc ||
      !inst->n_machines || !inst->first_stage || !inst->ready || !inst->due)
    return FFS_E_INVAL;
  hipLaunchKernelGGL(features_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, *inst, feats);
  return ok(hipGetLastError()) ? FFS_OK : FFS_E_DEVICE;
}

size_t sg_table_workspace_size(int32_t n_genes) {
  if (n_genes < 1 || n_genes > FFS_SG_MAX_GENES) return 0;
  return table_ws(nullptr, n_genes).total;
}

int sg_score_table(const ffs_surrogate *m, const float *feats, int32_t n, float *table,
                   void *workspace, size_t workspace_bytes, void *stream) {
  if (!m || !m->theta || !m->w2t_bf16 || !feats || !table || n < 1 || n > FFS_SG_MAX_GENES)
    return FFS_E_INVAL;
  const TableWs L = table_ws(workspace, n);
  if (!workspace || workspace_bytes < L.total) return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int Q = n * n;
  hipLaunchKernelGGL(ctab_kernel, dim3(grid1(n * H)), dim3(256), 0, s, (const float *)m->theta,
                     feats, n, L.ctab);
  hipLaunchKernelGGL(table_fwd_kernel<false>, dim3((Q + BM - 1) / BM, H / BN), dim3(256), 0, s,
                     (const float *)m->theta, (const float *)L.ctab,
                     (const uint16_t *)m->w2t_bf16, n, (float *)nullptr, L.r_part);
  hipLaunchKernelGGL(table_sum_kernel, dim3(grid1(Q)), dim3(256), 0, s, (const float *)L.r_part,
                     Q, table);
  return ok(hipGetLastError()) ? FFS_OK : FFS_E_DEVICE;
}

size_t sg_train_workspace_size(int32_t n_genes, int32_t batch) {
  if (n_genes < 1 || n_genes > FFS_SG_MAX_GENES || batch < 1 || batch > FFS_SG_MAX_BATCH) return 0;
  return train_ws(nullptr, n_genes, batch).total;
}

int sg_targets(const int64_t *obj, int32_t count, int32_t group, float *target, void *workspace,
               size_t workspace_bytes, void *stream) {
  if (!obj || !target || count < 0 || group < 1) return FFS_E_INVAL;
  if (!workspace || workspace_bytes < (size_t)kHeaderBytes) return FFS_E_WORKSPACE;
  if (count == 0) return FFS_OK;
  hipStream_t s = (hipStream_t)stream;
  int32_t *status = (int32_t *)workspace;
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, s, status);
  hipLaunchKernelGGL(targets_kernel, dim3((count + group - 1) / group), dim3(256), 0, s, obj,
                     count, group, target, status);
  return ok(hipGetLastError()) ? FFS_OK : FFS_E_DEVICE;
}

int sg_train_step(ffs_surrogate *m, const float *feats, int32_t n, const int32_t *prio,
                  const float *target, int32_t B, float lr, float *loss, float *grad,
                  void *workspace, size_t workspace_bytes, void *stream) {
  if (!m || !m->theta || !m->adam_m || !m->adam_v || !m->w2_bf16 || !m->w2t_bf16 || !feats ||
      !prio || !target || n < 1 || n > FFS_SG_MAX_GENES || B < 1 || B > FFS_SG_MAX_BATCH ||
      !(lr > 0.f) || m->step < 0)
    return FFS_E_INVAL;
  const TrainWs L = train_ws(workspace, n, B);
  if (!workspace || workspace_bytes < L.total) return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int Q = n * n, chunks = (Q + kChunk - 1) / kChunk, blocks = (Q + BM - 1) / BM;
  const int rchunks = (Q + kRowChunk - 1) / kRowChunk, dchunks = (B + kDChunk - 1) / kDChunk;
  const int hchunks = (B + kBatchChunk - 1) / kBatchChunk;
  const float *th = m->theta;
  const int32_t *st = L.status;
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(1), 0, s, L.status);
  hipLaunchKernelGGL(validate_kernel, dim3(grid1(B)), dim3(256), 0, s, prio, target, n, B,
                     L.status);
  hipLaunchKernelGGL(ctab_kernel, dim3(grid1(n * H)), dim3(256), 0, s, th, feats, n, L.ctab);
  hipLaunchKernelGGL(table_fwd_kernel<true>, dim3(blocks, H / BN), dim3(256), 0, s, th,
                     (const float *)L.ctab, (const uint16_t *)m->w2t_bf16, n, L.h2,
                     (float *)nullptr);
  hipLaunchKernelGGL(batch_fwd_kernel, dim3(B), dim3(64), 0, s, th, (const float *)L.h2, prio,
                     target, n, B, L.z, L.dy, L.sq, st);
  hipLaunchKernelGGL(dtable_kernel, dim3(n, dchunks), dim3(256), 0, s, prio, (const float *)L.dy,
                     n, B, L.Dpart, st);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid1(Q)), dim3(256), 0, s, (const float *)L.Dpart,
                     dchunks, (size_t)Q, Q, L.D, st);
  hipLaunchKernelGGL(head_kernel, dim3(hchunks), dim3(256), 0, s, (const float *)L.dy,
                     (const float *)L.z, (const float *)L.sq, B, L.head, st);
  hipLaunchKernelGGL(head_sum_kernel, dim3(1), dim3(256), 0, s, (const float *)L.head, hchunks, B,
                     L.grad, L.loss, st);
  hipLaunchKernelGGL(db2_part_kernel, dim3(rchunks), dim3(256), 0, s, th, (const float *)L.h2,
                     (const float *)L.D, n, L.part_b2, st);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(256), 0, s, (const float *)L.part_b2,
                     rchunks, (size_t)H, H, L.grad + kB2, st);
  hipLaunchKernelGGL(bwd_h1_kernel, dim3(blocks, H / BN), dim3(256), 0, s, th,
                     (const float *)L.ctab, feats, (const float *)L.h2, (const float *)L.D,
                     (const uint16_t *)m->w2_bf16, n, L.part1, st);
  hipLaunchKernelGGL(reduce_w1_kernel, dim3(grid1(5 * H)), dim3(256), 0, s,
                     (const float *)L.part1, blocks, L.grad, st);
  hipLaunchKernelGGL(bwd_w2_kernel, dim3(H / BM, H / BN, chunks), dim3(256), 0, s, th,
                     (const float *)L.ctab, (const float *)L.h2, (const float *)L.D, n,
                     L.part_w2, st);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid1(H * H)), dim3(256), 0, s,
                     (const float *)L.part_w2, chunks, (size_t)H * H, H * H, L.grad + kW2, st);
  if (!ok(hipGetLastError())) return FFS_E_DEVICE;
  if (grad && !ok(hipMemcpyAsync(grad, L.grad, sizeof(float) * FFS_SG_PARAMS,
                                 hipMemcpyDeviceToDevice, s)))
    return FFS_E_DEVICE;
  if (loss && !ok(hipMemcpyAsync(loss, L.loss, sizeof(float), hipMemcpyDeviceToDevice, s)))
    return FFS_E_DEVICE;
  const int t = m->step + 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
  hipLaunchKernelGGL(adam_kernel, dim3(grid1(FFS_SG_PARAMS)), dim3(256), 0, s, m->theta, m->adam_m,
                     m->adam_v, (const float *)L.grad, lr, c1, c2, m->w2_bf16, m->w2t_bf16, st);
  if (!ok(hipGetLastError())) return FFS_E_DEVICE;
  m->step = t;
  return FFS_OK;
}

}  // extern "C"
