// ffsga: gfx950 kernels and the C ABI for the EDFFS hybrid-GA hot path
// (Luo, Fujimura, El Baz, arXiv 1903.10741). The ABI is declared and
// documented in include/ffsga.h.
//
// Mapping onto CDNA4
//   * One wavefront (64 lanes) decodes one chromosome. The op loop of a decode
//     is serial (each placement changes the power profile the next one sees),
//     so the wave parallelises inside a placement: the lanes examine 64
//     consecutive profile slots at once and a ballot gives the slots that
//     would break the peak; the push-right then runs on that 64-bit mask in
//     scalar registers.
//   * The power profile is one byte per time slot (Q_max <= 255) in LDS, next
//     to the job order and per-job ready times of the chromosome. A decode
//     whose schedule outgrows the on-chip slots is redone by an overflow
//     kernel with the profile in global memory, sized by the instance's
//     horizon bound, so no schedule is ever cut short.
//   * Processing time and power of every (job, stage, machine) are packed in
//     one 32-bit word (P | Q << 16); a placement reads its row through the
//     scalar cache, and the earliest-completion machine choice runs on the
//     scalar unit.
//   * The GA generation is one launch: each wave selects its two parents from
//     the previous generation's objectives, builds its child (crossover,
//     correction, mutation) in LDS, writes it out and decodes it. A second
//     launch per island does the elitist replacement; migration adds two
//     launches every mig_interval generations.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "ffsga.h"

typedef unsigned long long u64;
typedef __attribute__((address_space(4))) const int32_t c_i32;
typedef __attribute__((address_space(4))) const uint32_t c_u32;
typedef __attribute__((address_space(4))) const int64_t c_i64;

namespace {

constexpr int kWave = 64;
constexpr int kMaxGenes = 4096;
constexpr int kMaxStages = 127;
constexpr int kDefaultLdsSlots = 8192;
constexpr int kFixBlocks = 64;       // overflow decodes in flight at once
constexpr int kHeaderBytes = 256;

// Device-side status word and small results at the head of every workspace.
struct Header {
  int32_t err;          // bit 0: invalid input, bit 1: infeasible power
  int32_t ovf_count;    // decodes waiting for the overflow kernel
  int32_t ovf_done;     // overflow blocks finished (last one resets)
  int32_t pad0;
  int64_t horizon;
  int64_t frozen_tardiness;
  int32_t frozen_cmax, n_running, n_active, pad1;
  unsigned long long work;  // algorithmic work of every decode of a GA
};
static_assert(sizeof(Header) <= kHeaderBytes, "header");

enum : int32_t { kErrInval = 1, kErrInfeasible = 2 };

__host__ __device__ constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): the counter-based generator every GA
// draw comes from, keyed (seed, shop), counter (individual, generation, event,
// purpose << 32 | block).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox(u64 c0, u64 c1, u64 c2, u64 c3, u64 k0, u64 k1, u64 out[4]) {
  const u64 m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
  const u64 w0 = 0x9E3779B97F4A7C15ull, w1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const u64 h0 = __umul64hi(m0, c0), l0 = m0 * c0;
    const u64 h1 = __umul64hi(m1, c2), l1 = m1 * c2;
    c0 = h1 ^ c1 ^ k0;
    c1 = l1;
    c2 = h0 ^ c3 ^ k1;
    c3 = l0;
    k0 += w0;
    k1 += w1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ uint32_t draw_below(u64 w, uint32_t n) {
  return (uint32_t)(((w >> 32) * (u64)n) >> 32);
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// ---------------------------------------------------------------------------
// Instance as the kernels see it.
// ---------------------------------------------------------------------------
struct DInst {
  const uint32_t *pq;        // [n_jobs][g][omp]: P | Q << 16
  const int32_t *nm;         // [g]
  const int32_t *due;        // [n_jobs]
  const int32_t *first;      // [n_jobs]
  const int32_t *ready;      // [n_jobs]
  const int32_t *mfree;      // [g][om]
  const int32_t *running;    // [nr][2]
  const int32_t *active;     // [n]
  int64_t frozen_t;
  int32_t n_jobs, g, om, omp, q_max, wt, rs, nr, n, frozen_cmax, horizon;
};

template <class T>
__device__ __forceinline__ T ld_const(const T *p, size_t i) {
  typedef __attribute__((address_space(4))) const T cT;
  return ((cT *)p)[i];
}

// Profile with one byte per slot in LDS.
struct LdsProfile {
  uint8_t *p;
  int cap;
  __device__ void clear() const {
    uint32_t *w = (uint32_t *)p;
    for (int x = __lane_id(); x < cap / 4; x += kWave) w[x] = 0;
  }
  __device__ uint32_t get(int x) const { return p[x]; }
  __device__ void add(int x, uint32_t q) const {
    atomicAdd((uint32_t *)(p + (x & ~3)), q << (8 * (x & 3)));
  }
  __device__ void order() const { __asm__ volatile("" ::: "memory"); }
};

// Profile with one byte per slot in global memory (overflow tier).
struct GlobalProfile {
  uint8_t *p;
  int cap;
  __device__ void clear() const {
    uint32_t *w = (uint32_t *)p;
    for (int x = __lane_id(); x < (cap + 3) / 4; x += kWave)
      __hip_atomic_store(w + x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  __device__ uint32_t get(int x) const {
    uint32_t w = __hip_atomic_load((uint32_t *)(p + (x & ~3)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    return (w >> (8 * (x & 3))) & 0xFFu;
  }
  __device__ void add(int x, uint32_t q) const {
    atomicAdd((uint32_t *)(p + (x & ~3)), q << (8 * (x & 3)));
  }
  __device__ void order() const { __threadfence(); }
};

enum : int { kDecOk = 0, kDecOverflow = 1, kDecInval = 2, kDecInfeasible = 3 };

// Decode the chromosome in gene[0..n) (LDS) with the profile `prof`.
// order[] is LDS scratch of n int2. On kDecOk, *obj_out holds eq. (1).
// Every lane must call this; results are uniform.
template <int MAXM, class Prof>
__device__ int decode_core(const DInst &I, const int32_t *gene, int2 *order, const Prof &prof,
                           int64_t *obj_out, int64_t *work_out, int32_t *start_out,
                           int32_t *mach_out) {
  const int lane = __lane_id();
  const int n = I.n;
  // Job order: the job of gene k has rank n - prio_k (larger priority first).
  for (int x = lane; x < n; x += kWave) order[x].x = -1;
  int bad = 0;
  for (int k = lane; k < n; k += kWave) {
    const int v = gene[k];
    if (v >= 1 && v <= n) order[n - v].x = k;
    else bad = 1;
  }
  __asm__ volatile("" ::: "memory");
  for (int x = lane; x < n; x += kWave) {
    const int k = order[x].x;
    if (k < 0) {
      bad = 1;
    } else {
      const int j = ld_const(I.active, k);
      order[x] = make_int2(j | (ld_const(I.first, j) << 24), ld_const(I.ready, j));
    }
  }
  if (__ballot(bad)) return kDecInval;

  // Power held by the ops running at RS, on [RS, end).
  prof.clear();
  prof.order();
  for (int r = 0; r < I.nr; ++r) {
    const int len = ld_const(I.running, 2 * r) - I.rs;
    const uint32_t q = (uint32_t)ld_const(I.running, 2 * r + 1);
    if (len > prof.cap) return kDecOverflow;
    for (int x = lane; x < len; x += kWave) prof.add(x, q);
  }
  prof.order();

  const int rs = I.rs, cap = prof.cap;
  int64_t tard = I.frozen_t, work = 0;
  int cmax = I.frozen_cmax;
  for (int s = 0; s < I.g; ++s) {
    const int os = ld_const(I.nm, s);
    int fr[MAXM];
#pragma unroll
    for (int m = 0; m < MAXM; ++m) fr[m] = m < os ? ld_const(I.mfree, (size_t)s * I.om + m) : 0;
    for (int x = 0; x < n; ++x) {
      const int2 pi = order[x];
      const int jf = uni(pi.x), rdy = uni(pi.y);
      const int j = jf & 0xFFFFFF;
      if ((jf >> 24) > s) continue;  // frozen at this stage
      const int est = max(rs, rdy);
      const size_t row = ((size_t)j * I.g + s) * I.omp;
      // Machine of earliest completion, ties to the lowest index. The packed
      // row is padded to MAXM words, so it is read whole.
      uint32_t rowv[MAXM];
#pragma unroll
      for (int m = 0; m < MAXM; ++m) rowv[m] = ld_const(I.pq, row + m);
      int best = INT_MAX, mb = 0, first = 0;
      uint32_t pq = 0;
#pragma unroll
      for (int m = 0; m < MAXM; ++m) {
        const int a = max(est, fr[m]);
        const int e = a + (int)(rowv[m] & 0xFFFFu);
        if (m < os && e < best) {
          best = e;
          mb = m;
          pq = rowv[m];
          first = a;
        }
      }
      const int p = (int)(pq & 0xFFFFu), q = (int)(pq >> 16);
      if (q > I.q_max) return kDecInfeasible;
      const uint32_t thr = (uint32_t)(I.q_max - q);
      // Push right: earliest t >= t0 with every slot of [t, t+p) at most thr.
      // [t, scan) is known clean; the lanes read [scan, scan+64) and the
      // window jumps past the last breaking slot inside it.
      const int t0 = first - rs;
      int t = t0, scan = t0;
      while (scan < t + p) {
        const int xx = scan + lane;
        const uint32_t v = xx < cap ? prof.get(xx) : 0u;
        const u64 over = __ballot(v > thr);
        for (;;) {
          const int lo = max(t - scan, 0);  // window start inside this chunk
          if (lo >= kWave) {
            scan = t;
            break;
          }
          const int hi = min(kWave, t + p - scan);
          const u64 mask = (hi >= kWave ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
          const u64 hit = over & mask;
          if (!hit) {
            scan += hi;
            break;
          }
          t = scan + (kWave - __clzll(hit));
        }
      }
      if (t + p > cap) return kDecOverflow;
      for (int b = lane; b < p; b += kWave) prof.add(t + b, (uint32_t)q);
      prof.order();
      const int end = t + p + rs;
#pragma unroll
      for (int m = 0; m < MAXM; ++m) fr[m] = m == mb ? end : fr[m];
      if (lane == 0) {
        order[x].y = end;
        if (start_out) {
          start_out[(size_t)j * I.g + s] = t + rs;
          mach_out[(size_t)j * I.g + s] = mb;
        }
      }
      if (s == I.g - 1) {
        const int late = end - ld_const(I.due, j);
        tard += late > 0 ? late : 0;
        cmax = max(cmax, end);
      }
      work += 3 * os + (t - t0) + 2 * p;
    }
  }
  if (lane == 0) {
    *obj_out = (int64_t)I.wt * tard + cmax;
    if (work_out) *work_out = work;
  }
  return kDecOk;
}

struct Lds {
  int32_t *gene;
  int2 *order;
  uint8_t *prof;
};

__device__ __forceinline__ Lds carve_lds(uint8_t *smem, int n) {
  Lds l;
  l.gene = (int32_t *)smem;
  l.order = (int2 *)(smem + align_up((size_t)4 * n + 4, 16));
  l.prof = smem + align_up((size_t)4 * n + 4, 16) + align_up((size_t)8 * n + 16, 16);
  return l;
}

__host__ __device__ inline size_t lds_bytes(int n, int cap) {
  return align_up((size_t)4 * n + 4, 16) + align_up((size_t)8 * n + 16, 16) + align_up(cap, 16);
}

__device__ void flag_error(Header *h, int status) {
  if (__lane_id() == 0) atomicOr(&h->err, status == kDecInfeasible ? kErrInfeasible : kErrInval);
}

__device__ void push_overflow(Header *h, int32_t *list, int idx) {
  if (__lane_id() != 0) return;
  if (!list) {  // the host sized the profile to the horizon bound: cannot happen
    atomicOr(&h->err, kErrInval);
    return;
  }
  const int e = atomicAdd(&h->ovf_count, 1);
  list[e] = idx;
}

// ---------------------------------------------------------------------------
// Population decode (ffs_decode).
// ---------------------------------------------------------------------------
template <int MAXM>
__global__ __launch_bounds__(64) void decode_kernel(DInst I, const int32_t *__restrict__ prio,
                                                    int64_t *obj, int64_t *work, int32_t *start,
                                                    int32_t *mach, Header *hdr, int32_t *ovf_list,
                                                    int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x;
  Lds l = carve_lds(smem, I.n);
  const int32_t *src = prio + (size_t)i * I.n;
  for (int k = __lane_id(); k < I.n; k += kWave) l.gene[k] = src[k];
  __asm__ volatile("" ::: "memory");
  const size_t plan = (size_t)i * I.n_jobs * I.g;
  const int st = decode_core<MAXM>(I, l.gene, l.order, LdsProfile{l.prof, cap}, obj + i,
                                   work ? work + i : nullptr, start ? start + plan : nullptr,
                                   mach ? mach + plan : nullptr);
  if (st == kDecOk) return;
  if (__lane_id() == 0) obj[i] = -1;
  if (st == kDecOverflow) push_overflow(hdr, ovf_list, i);
  else flag_error(hdr, st);
}

// Redo the decodes listed as overflowed with a global-memory profile of
// `horizon` slots per block; the last block to finish clears the list.
template <int MAXM>
__global__ __launch_bounds__(64) void overflow_kernel(DInst I, const int32_t *__restrict__ prio,
                                                      int64_t *obj, int64_t *work, int32_t *start,
                                                      int32_t *mach, Header *hdr,
                                                      const int32_t *ovf_list, uint8_t *gprof,
                                                      size_t gstride) {
  extern __shared__ __align__(16) uint8_t smem[];
  Lds l = carve_lds(smem, I.n);
  const int count = __hip_atomic_load(&hdr->ovf_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const GlobalProfile prof{gprof + gstride * blockIdx.x, I.horizon};
  for (int e = blockIdx.x; e < count; e += gridDim.x) {
    const int i = uni(ovf_list[e]);
    const int32_t *src = prio + (size_t)i * I.n;
    for (int k = __lane_id(); k < I.n; k += kWave) l.gene[k] = src[k];
    __asm__ volatile("" ::: "memory");
    const size_t plan = (size_t)i * I.n_jobs * I.g;
    int64_t w = 0;
    const int st = decode_core<MAXM>(I, l.gene, l.order, prof, obj + i, work ? work + i : &w,
                                     start ? start + plan : nullptr, mach ? mach + plan : nullptr);
    if (st == kDecOk && !work && __lane_id() == 0) atomicAdd(&hdr->work, (unsigned long long)w);
    if (st != kDecOk) {
      if (__lane_id() == 0) obj[i] = -1;
      flag_error(hdr, st == kDecOverflow ? kDecInval : st);
    }
  }
  __threadfence();
  if (__lane_id() == 0) {
    const int done = atomicAdd(&hdr->ovf_done, 1);
    if (done == (int)gridDim.x - 1) {
      __hip_atomic_store(&hdr->ovf_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&hdr->ovf_done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// GA kernels (Section 4.4).
// ---------------------------------------------------------------------------
struct GaDev {
  const int32_t *prio_in;
  const int64_t *obj_in;
  int32_t *prio_out;
  int64_t *obj_out;
  int32_t *elite;
  int64_t *elite_obj;
  int32_t *stage_prio;   // migration staging [islands][mig_k][n]
  int64_t *stage_obj;    // [islands][mig_k]
  Header *hdr;
  int32_t *ovf_list;
  u64 seed, shop;
  int32_t event, rows, cols, islands, mig_k;
  uint32_t pc, pm;
};

// Local selection (Fig. 9 is not available; reading: the slot and its four
// torus neighbours within the island, order self, up, down, left, right,
// lowest objective wins, first on ties).
__device__ __forceinline__ int select_winner(const GaDev &A, int i) {
  const int K = A.rows * A.cols, base = i / K * K, loc = i % K;
  const int r = loc / A.cols, c = loc % A.cols;
  const int cand[5] = {i, base + ((r + A.rows - 1) % A.rows) * A.cols + c,
                       base + ((r + 1) % A.rows) * A.cols + c,
                       base + r * A.cols + (c + A.cols - 1) % A.cols,
                       base + r * A.cols + (c + 1) % A.cols};
  int w = cand[0];
  int64_t wo = ld_const(A.obj_in, (size_t)w);
#pragma unroll
  for (int k = 1; k < 5; ++k) {
    const int64_t o = ld_const(A.obj_in, (size_t)cand[k]);
    if (o < wo) {
      wo = o;
      w = cand[k];
    }
  }
  return w;
}

// Correction (Fig. 11): first occurrences stay; later duplicates take the
// values missing from 1..n in ascending order, in scan order.
// first_pos: LDS [n + 1], miss: LDS [n].
__device__ void correct_lds(int32_t *gene, int n, int32_t *first_pos, int32_t *miss) {
  const int lane = __lane_id();
  for (int v = lane; v <= n; v += kWave) first_pos[v] = INT_MAX;
  __asm__ volatile("" ::: "memory");
  for (int k = lane; k < n; k += kWave) {
    const int v = gene[k];
    if (v >= 1 && v <= n) atomicMin(&first_pos[v], k);
  }
  __asm__ volatile("" ::: "memory");
  const u64 below = (1ull << lane) - 1;
  int rank = 0;
  for (int b = 0; b < n; b += kWave) {
    const int v = b + lane + 1;
    const bool missing = v <= n && first_pos[v] == INT_MAX;
    const u64 m = __ballot(missing);
    if (missing) miss[rank + __popcll(m & below)] = v;
    rank += __popcll(m);
  }
  __asm__ volatile("" ::: "memory");
  rank = 0;
  for (int b = 0; b < n; b += kWave) {
    const int k = b + lane;
    const int v = k < n ? gene[k] : 1;
    const bool dup = k < n && (v < 1 || v > n || first_pos[v] != k);
    const u64 m = __ballot(dup);
    if (dup) gene[k] = miss[rank + __popcll(m & below)];
    rank += __popcll(m);
  }
  __asm__ volatile("" ::: "memory");
}

// Slot of block b. With a multiple of 8 islands the blocks of one island run
// on one XCD (blocks are dealt to the 8 XCDs round robin), so parents, written
// by the previous generation on the same XCD, come from its L2.
__device__ __forceinline__ int slot_of_block(int b, int K, int islands) {
  if (islands % 8 != 0) return b;
  const int xcd = b % 8, t = b / 8;
  return ((t / K) * 8 + xcd) * K + t % K;
}

template <int MAXM>
__global__ __launch_bounds__(64) void ga_generation_kernel(DInst I, GaDev A, int gen, int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = __lane_id();
  const int n = I.n, K = A.rows * A.cols;
  const int i = slot_of_block(blockIdx.x, K, A.islands);
  Lds l = carve_lds(smem, n);
  int32_t *first_pos = (int32_t *)l.order;
  int32_t *miss = first_pos + (n + 1);

  // Pair (Fig. 10 is not available; reading: horizontal neighbours
  // (r,2c)-(r,2c+1) on odd generations, vertical (2r,c)-(2r+1,c) on even).
  const int loc = i % K, r = loc / A.cols, c = loc % A.cols;
  int lead = -1, partner = -1;
  if (gen & 1) {
    if ((c | 1) < A.cols) {
      lead = i - (c & 1);
      partner = (c & 1) ? i - 1 : i + 1;
    }
  } else if ((r | 1) < A.rows) {
    lead = i - (r & 1) * A.cols;
    partner = (r & 1) ? i - A.cols : i + A.cols;
  }
  const int w_self = select_winner(A, i);
  const int32_t *mine = A.prio_in + (size_t)w_self * n;
  bool cross = false;
  int cut = n;
  if (lead >= 0 && n >= 2) {
    u64 w[4];
    philox((u64)lead, (u64)gen, (u64)A.event, 1ull << 32, A.seed, A.shop, w);
    cross = (uint32_t)(w[0] >> 32) < A.pc;
    cut = 1 + (int)draw_below(w[1], (uint32_t)(n - 1));
  }
  if (cross) {
    const int32_t *other = A.prio_in + (size_t)select_winner(A, partner) * n;
    for (int k = lane; k < n; k += kWave) l.gene[k] = k < cut ? mine[k] : other[k];
    __asm__ volatile("" ::: "memory");
    correct_lds(l.gene, n, first_pos, miss);
  } else {
    for (int k = lane; k < n; k += kWave) l.gene[k] = mine[k];
    __asm__ volatile("" ::: "memory");
  }
  if (n >= 2) {  // swap mutation (Fig. 12)
    u64 w[4];
    philox((u64)i, (u64)gen, (u64)A.event, 2ull << 32, A.seed, A.shop, w);
    if ((uint32_t)(w[0] >> 32) < A.pm) {
      const int x = (int)draw_below(w[1], (uint32_t)n);
      int y = (int)draw_below(w[2], (uint32_t)(n - 1));
      y += y >= x;
      if (lane == 0) {
        const int gx = l.gene[x];
        l.gene[x] = l.gene[y];
        l.gene[y] = gx;
      }
      __asm__ volatile("" ::: "memory");
    }
  }
  int32_t *dst = A.prio_out + (size_t)i * n;
  for (int k = lane; k < n; k += kWave) dst[k] = l.gene[k];
  int64_t work = 0;
  const int st = decode_core<MAXM>(I, l.gene, l.order, LdsProfile{l.prof, cap}, A.obj_out + i,
                                   &work, nullptr, nullptr);
  if (st == kDecOk) {
    if (lane == 0) atomicAdd(&A.hdr->work, (unsigned long long)work);
    return;
  }
  if (lane == 0) A.obj_out[i] = -1;
  if (st == kDecOverflow) push_overflow(A.hdr, A.ovf_list, i);
  else flag_error(A.hdr, st);
}

// Generation 0: Fisher-Yates over 1..n, draw d from word d % 4 of block d / 4
// of purpose 0, then decode.
template <int MAXM>
__global__ __launch_bounds__(64) void ga_init_kernel(DInst I, GaDev A, int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = __lane_id();
  const int n = I.n, i = blockIdx.x;
  Lds l = carve_lds(smem, n);
  uint32_t *hi = (uint32_t *)l.order;  // n - 1 high words
  for (int k = lane; k < n; k += kWave) l.gene[k] = k + 1;
  const int n_blocks = (n - 1 + 3) / 4;
  for (int b = lane; b < n_blocks; b += kWave) {
    u64 w[4];
    philox((u64)i, 0ull, (u64)A.event, (u64)b, A.seed, A.shop, w);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * b + k < n - 1) hi[4 * b + k] = (uint32_t)(w[k] >> 32);
  }
  __asm__ volatile("" ::: "memory");
  if (lane == 0) {
    for (int pos = n - 1; pos >= 1; --pos) {
      const int r = (int)(((u64)hi[n - 1 - pos] * (u64)(pos + 1)) >> 32);
      const int t = l.gene[pos];
      l.gene[pos] = l.gene[r];
      l.gene[r] = t;
    }
  }
  __asm__ volatile("" ::: "memory");
  int32_t *dst = A.prio_out + (size_t)i * n;
  for (int k = lane; k < n; k += kWave) dst[k] = l.gene[k];
  int64_t work = 0;
  const int st = decode_core<MAXM>(I, l.gene, l.order, LdsProfile{l.prof, cap}, A.obj_out + i,
                                   &work, nullptr, nullptr);
  if (st == kDecOk) {
    if (lane == 0) atomicAdd(&A.hdr->work, (unsigned long long)work);
    return;
  }
  if (lane == 0) A.obj_out[i] = -1;
  if (st == kDecOverflow) push_overflow(A.hdr, A.ovf_list, i);
  else flag_error(A.hdr, st);
}

// Block-wide (value, index) reductions with the lowest index on ties.
template <bool MAX>
__device__ void block_arg(int64_t v, int idx, int64_t *sv, int *si, int64_t &out_v, int &out_i) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = idx;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      const int64_t a = sv[t], b = sv[t + h];
      const int ia = si[t], ib = si[t + h];
      const bool take_b = MAX ? (b > a || (b == a && ib < ia)) : (b < a || (b == a && ib < ia));
      if (take_b) {
        sv[t] = b;
        si[t] = ib;
      }
    }
    __syncthreads();
  }
  out_v = sv[0];
  out_i = si[0];
  __syncthreads();
}

template <bool MAX>
__device__ void island_arg(const int64_t *obj, int base, int K, const uint8_t *taken, int64_t *sv,
                           int *si, int64_t &out_v, int &out_i) {
  int64_t bv = MAX ? LLONG_MIN : LLONG_MAX;
  int bi = INT_MAX;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    if (taken && taken[k]) continue;
    const int64_t o = obj[base + k];
    if (MAX ? (o > bv || (o == bv && k < bi)) : (o < bv || (o == bv && k < bi))) {
      bv = o;
      bi = k;
    }
  }
  block_arg<MAX>(bv, bi, sv, si, out_v, out_i);
}

// Elitist replacement (Section 4.4): the island's best child refreshes the
// best-in-history, which then overwrites the island's worst child.
__global__ __launch_bounds__(256) void replace_kernel(int32_t *prio, int64_t *obj, int32_t *elite,
                                                      int64_t *elite_obj, int K, int n) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  const int I = blockIdx.x, base = I * K;
  int64_t bv, wv;
  int b, w;
  island_arg<false>(obj, base, K, nullptr, sv, si, bv, b);
  island_arg<true>(obj, base, K, nullptr, sv, si, wv, w);
  if (bv < elite_obj[I]) {
    for (int k = threadIdx.x; k < n; k += blockDim.x)
      elite[(size_t)I * n + k] = prio[(size_t)(base + b) * n + k];
    __syncthreads();
    if (threadIdx.x == 0) elite_obj[I] = bv;
    __syncthreads();
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    prio[(size_t)(base + w) * n + k] = elite[(size_t)I * n + k];
  if (threadIdx.x == 0) obj[base + w] = elite_obj[I];
}

__global__ __launch_bounds__(256) void elite_init_kernel(const int32_t *prio, const int64_t *obj,
                                                         int32_t *elite, int64_t *elite_obj, int K,
                                                         int n) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  const int I = blockIdx.x, base = I * K;
  int64_t bv;
  int b;
  island_arg<false>(obj, base, K, nullptr, sv, si, bv, b);
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    elite[(size_t)I * n + k] = prio[(size_t)(base + b) * n + k];
  if (threadIdx.x == 0) elite_obj[I] = bv;
}

// Ring migration (Section 4.4; Fig. 13 not available). Reading: snapshot the
// mig_k best of every island (by objective, then slot), then island i's mig_k
// worst (by objective descending, then slot) take island i-1's best in order;
// an immigrant better than the elite becomes the elite.
__global__ __launch_bounds__(256) void migrate_collect_kernel(const int32_t *prio, const int64_t *obj,
                                                              int32_t *stage_prio, int64_t *stage_obj,
                                                              int K, int n, int mig_k) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  const int I = blockIdx.x, base = I * K;
  for (int k = threadIdx.x; k < K; k += blockDim.x) taken[k] = 0;
  __syncthreads();
  for (int r = 0; r < mig_k; ++r) {
    int64_t bv;
    int b;
    island_arg<false>(obj, base, K, taken, sv, si, bv, b);
    for (int k = threadIdx.x; k < n; k += blockDim.x)
      stage_prio[((size_t)I * mig_k + r) * n + k] = prio[(size_t)(base + b) * n + k];
    if (threadIdx.x == 0) {
      stage_obj[I * mig_k + r] = bv;
      taken[b] = 1;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void migrate_apply_kernel(int32_t *prio, int64_t *obj,
                                                            int32_t *elite, int64_t *elite_obj,
                                                            const int32_t *stage_prio,
                                                            const int64_t *stage_obj, int K, int n,
                                                            int mig_k, int islands) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  const int I = blockIdx.x, base = I * K, src = (I + islands - 1) % islands;
  for (int k = threadIdx.x; k < K; k += blockDim.x) taken[k] = 0;
  __syncthreads();
  for (int r = 0; r < mig_k; ++r) {
    int64_t wv;
    int w;
    island_arg<true>(obj, base, K, taken, sv, si, wv, w);
    if (threadIdx.x == 0) taken[w] = 1;
    const int64_t io = stage_obj[src * mig_k + r];
    const int32_t *ip = stage_prio + ((size_t)src * mig_k + r) * n;
    for (int k = threadIdx.x; k < n; k += blockDim.x) prio[(size_t)(base + w) * n + k] = ip[k];
    if (threadIdx.x == 0) obj[base + w] = io;
    __syncthreads();
    if (io < elite_obj[I]) {
      for (int k = threadIdx.x; k < n; k += blockDim.x) elite[(size_t)I * n + k] = ip[k];
      __syncthreads();
      if (threadIdx.x == 0) elite_obj[I] = io;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void best_kernel(const int32_t *elite, const int64_t *elite_obj,
                                                   int islands, int n, int32_t *prio_out,
                                                   int64_t *obj_out) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  int64_t bv = LLONG_MAX;
  int bi = INT_MAX;
  for (int k = threadIdx.x; k < islands; k += blockDim.x)
    if (elite_obj[k] < bv || (elite_obj[k] == bv && k < bi)) {
      bv = elite_obj[k];
      bi = k;
    }
  block_arg<false>(bv, bi, sv, si, bv, bi);
  for (int k = threadIdx.x; k < n; k += blockDim.x) prio_out[k] = elite[(size_t)bi * n + k];
  if (threadIdx.x == 0) *obj_out = bv;
}

// ---------------------------------------------------------------------------
// Instance preparation: packing, checks, horizon bound, rescheduling.
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const int32_t *proc, const int32_t *power, uint32_t *pq, int rows,
                            int om, int omp) {
  const size_t total = (size_t)rows * omp;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (size_t)gridDim.x * blockDim.x) {
    const size_t row = x / omp;
    const int m = (int)(x % omp);
    uint32_t v = 0;
    if (m < om) {
      const uint32_t p = (uint32_t)proc[row * om + m] & 0xFFFFu;
      const uint32_t q = (uint32_t)power[row * om + m] & 0xFFFFu;
      v = p | (q << 16);
    }
    pq[x] = v;
  }
}

struct PrepArgs {
  const int32_t *nm, *proc, *power, *first, *ready, *mfree, *running, *active;
  int32_t n_jobs, g, om, q_max, rs, nr, n;
};

__device__ void block_reduce_i64(int64_t v, int64_t *sh, bool is_max, int64_t &out) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) sh[t] = is_max ? max(sh[t], sh[t + h]) : sh[t] + sh[t + h];
    __syncthreads();
  }
  out = sh[0];
  __syncthreads();
}

// Checks and the horizon bound of an instance (one block of 1024 threads).
// Every start is at most max(earliest start, machine free, end of the latest
// op placed so far), since past that only ops running at RS (ending by
// `base`) use power; so every end is within base + the sum over unfrozen ops
// of their longest processing time.
__device__ void prepare_body(const PrepArgs &a, Header *h) {
  __shared__ int64_t sh[1024];
  int err = 0;
  int64_t base = a.rs, sum = 0;
  int unfrozen = 0;
  for (int s = threadIdx.x; s < a.g; s += blockDim.x)
    if (a.nm[s] < 1 || a.nm[s] > a.om) err |= kErrInval;
  for (int j = threadIdx.x; j < a.n_jobs; j += blockDim.x) {
    const int f = a.first[j];
    if (f < 0 || f > a.g) err |= kErrInval;
    unfrozen += f < a.g;
  }
  for (int k = threadIdx.x; k < a.n; k += blockDim.x) {
    const int j = a.active[k];
    if (j < 0 || j >= a.n_jobs || (k > 0 && a.active[k - 1] >= j)) {
      err |= kErrInval;
      continue;
    }
    const int f = a.first[j];
    if (f < 0 || f >= a.g) {
      err |= kErrInval;
      continue;
    }
    base = max(base, (int64_t)a.ready[j]);
    for (int s = f; s < a.g; ++s) {
      const int os = min(max(a.nm[s], 1), a.om);
      int pmax = 0;
      for (int m = 0; m < os; ++m) {
        const int p = a.proc[((size_t)j * a.g + s) * a.om + m];
        const int q = a.power[((size_t)j * a.g + s) * a.om + m];
        if (p < 1 || p > 65535 || q < 1 || q > 65535) err |= kErrInval;
        if (q > a.q_max) err |= kErrInfeasible;
        pmax = max(pmax, p);
      }
      sum += pmax;
    }
  }
  for (int x = threadIdx.x; x < a.g * a.om; x += blockDim.x)
    if (x % a.om < a.nm[x / a.om]) base = max(base, (int64_t)a.mfree[x]);
  for (int r = threadIdx.x; r < a.nr; r += blockDim.x) base = max(base, (int64_t)a.running[2 * r]);
  int64_t tot_base, tot_sum, tot_unfrozen;
  block_reduce_i64(base, sh, true, tot_base);
  block_reduce_i64(sum, sh, false, tot_sum);
  block_reduce_i64(unfrozen, sh, false, tot_unfrozen);
  if (err) atomicOr(&h->err, err);
  if (threadIdx.x == 0) {
    if (tot_unfrozen != a.n) atomicOr(&h->err, kErrInval);
    h->horizon = tot_base - a.rs + tot_sum + 1;
  }
}

__global__ __launch_bounds__(1024) void prepare_kernel(PrepArgs a, Header *h) { prepare_body(a, h); }

struct ReschedArgs {
  // previous instance
  const int32_t *nm, *proc, *power, *release, *due;
  int32_t n0, g, om, q_max, prev_rs;
  const int32_t *plan_start, *plan_mach;
  int32_t rs, n_new;
  const int32_t *new_proc, *new_power, *new_release, *new_due;
  // next instance
  int32_t *proc_o, *power_o, *release_o, *due_o, *first_o, *ready_o, *mfree_o, *running_o,
      *active_o;
  int32_t running_cap;  // pairs of room in running_o
};

// Predictive-reactive rescheduling (Section 4.1) in one block of 1024
// threads: freeze ops started before rs (eq. (10)); an op running at rs
// (S < rs < S + P, Algorithm 1) keeps its machine and power until it ends.
__global__ __launch_bounds__(1024) void reschedule_kernel(ReschedArgs a, Header *h) {
  __shared__ int64_t sh[1024];
  __shared__ int scan_run[1024], scan_act[1024];
  __shared__ int carry_run, carry_act;
  const int t = threadIdx.x, T = blockDim.x;
  const int g = a.g, om = a.om, n = a.n0 + a.n_new;
  const size_t row = (size_t)g * om;
  for (size_t x = t; x < (size_t)a.n0 * row; x += T) {
    a.proc_o[x] = a.proc[x];
    a.power_o[x] = a.power[x];
  }
  for (size_t x = t; x < (size_t)a.n_new * row; x += T) {
    a.proc_o[(size_t)a.n0 * row + x] = a.new_proc[x];
    a.power_o[(size_t)a.n0 * row + x] = a.new_power[x];
  }
  for (int j = t; j < a.n0; j += T) {
    a.release_o[j] = a.release[j];
    a.due_o[j] = a.due[j];
  }
  for (int j = t; j < a.n_new; j += T) {
    a.release_o[a.n0 + j] = a.new_release[j];
    a.due_o[a.n0 + j] = a.new_due[j];
  }
  for (int x = t; x < g * om; x += T) a.mfree_o[x] = 0;
  if (t == 0) {
    carry_run = 0;
    carry_act = 0;
  }
  __syncthreads();
  int err = 0;
  int64_t tard = 0, cmax = 0;
  for (int b0 = 0; b0 < n; b0 += T) {
    const int j = b0 + t;
    int run = 0, act = 0, run_end = 0, run_q = 0;
    if (j < a.n0) {
      int f = g;
      for (int s = 0; s < g; ++s)
        if (a.plan_start[(size_t)j * g + s] >= a.rs) {
          f = s;
          break;
        }
      for (int s = f; s < g; ++s)
        if (a.plan_start[(size_t)j * g + s] < a.rs) err |= kErrInval;
      int last_end = a.release[j];
      for (int s = 0; s < f; ++s) {
        const int m = a.plan_mach[(size_t)j * g + s];
        if (m < 0 || m >= a.nm[s]) {
          err |= kErrInval;
          break;
        }
        const int st = a.plan_start[(size_t)j * g + s];
        const int end = st + a.proc[((size_t)j * g + s) * om + m];
        atomicMax(&a.mfree_o[s * om + m], end);
        if (end > a.rs) {
          run = 1;
          run_end = end;
          run_q = a.power[((size_t)j * g + s) * om + m];
        }
        last_end = end;
      }
      a.first_o[j] = f;
      a.ready_o[j] = f == 0 ? a.release[j] : last_end;
      act = f < g;
      if (f == g) {
        tard += max(last_end - a.due[j], 0);
        cmax = max(cmax, (int64_t)last_end);
      }
    } else if (j < n) {
      a.first_o[j] = 0;
      a.ready_o[j] = a.new_release[j - a.n0];
      act = 1;
    }
    // ordered compaction of running ops and active jobs (ascending job id)
    scan_run[t] = run;
    scan_act[t] = act;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {
      const int vr = t >= d ? scan_run[t - d] : 0, va = t >= d ? scan_act[t - d] : 0;
      __syncthreads();
      scan_run[t] += vr;
      scan_act[t] += va;
      __syncthreads();
    }
    if (run) {
      const int pos = carry_run + scan_run[t] - 1;
      if (pos < a.running_cap) {
        a.running_o[2 * pos] = run_end;
        a.running_o[2 * pos + 1] = run_q;
      } else {
        err |= kErrInval;  // more ops running at rs than machines: the plan overlaps
      }
    }
    if (act) a.active_o[carry_act + scan_act[t] - 1] = j;
    __syncthreads();
    if (t == T - 1) {
      carry_run += scan_run[t];
      carry_act += scan_act[t];
    }
    __syncthreads();
  }
  int64_t tot_tard, tot_cmax;
  block_reduce_i64(tard, sh, false, tot_tard);
  block_reduce_i64(cmax, sh, true, tot_cmax);
  if (err) atomicOr(&h->err, err);
  if (t == 0) {
    h->frozen_tardiness = tot_tard;
    h->frozen_cmax = (int32_t)tot_cmax;
    h->n_running = carry_run;
    h->n_active = carry_act;
  }
  __threadfence_block();
  __syncthreads();
  PrepArgs p{a.nm, a.proc_o, a.power_o, a.first_o, a.ready_o, a.mfree_o, a.running_o, a.active_o,
             n, g, om, a.q_max, a.rs, min(carry_run, a.running_cap), carry_act};
  prepare_body(p, h);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> ev[4];
  size_t used[4] = {0, 0, 0, 0};
  double ms[4] = {0, 0, 0, 0};
  int64_t launches[4] = {0, 0, 0, 0};
};
Timing g_timing;
constexpr size_t kTimingPairs = 4096;

void drain_family(int f, size_t upto) {
  for (size_t k = 0; k < upto; ++k) {
    float ms = 0;
    (void)hipEventSynchronize(g_timing.ev[f][2 * k + 1]);
    (void)hipEventElapsedTime(&ms, g_timing.ev[f][2 * k], g_timing.ev[f][2 * k + 1]);
    g_timing.ms[f] += ms;
  }
}

template <typename K, typename... Args>
hipError_t launch(int family, K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t stream,
                  Args... args) {
  if (grid.x == 0) return hipSuccess;
  if (family >= 0 && g_timing.on) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (g_timing.used[family] == kTimingPairs) {
      drain_family(family, kTimingPairs);
      g_timing.used[family] = 0;
    }
    const size_t k = g_timing.used[family]++;
    g_timing.launches[family]++;
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)shmem, stream, g_timing.ev[family][2 * k],
                          g_timing.ev[family][2 * k + 1], 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, args...);
  }
  return hipGetLastError();
}

int max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

int omp_of(int om) { return om <= 8 ? 8 : 16; }

int check_host(const ffs_instance *in) {
  if (!in) return FFS_E_INVAL;
  if (in->n_stages < 1 || in->o_max < 1 || in->n_jobs < 0 || in->n_active < 0 ||
      in->n_active > in->n_jobs || in->n_running < 0 || in->q_max < 1)
    return FFS_E_INVAL;
  if (in->o_max > 16 || in->n_stages > kMaxStages || in->n_jobs >= (1 << 24) || in->q_max > 255 ||
      in->n_active > kMaxGenes)
    return FFS_E_UNSUPPORTED;
  if (!in->n_machines || !in->proc || !in->power || !in->due || !in->first_stage || !in->ready ||
      !in->machine_free || (in->n_running && !in->running) || (in->n_active && !in->active))
    return FFS_E_INVAL;
  return FFS_OK;
}

DInst make_dinst(const ffs_instance *in, const uint32_t *pq) {
  DInst d;
  d.pq = pq;
  d.nm = in->n_machines;
  d.due = in->due;
  d.first = in->first_stage;
  d.ready = in->ready;
  d.mfree = in->machine_free;
  d.running = in->running;
  d.active = in->active;
  d.frozen_t = in->frozen_tardiness;
  d.n_jobs = in->n_jobs;
  d.g = in->n_stages;
  d.om = in->o_max;
  d.omp = omp_of(in->o_max);
  d.q_max = in->q_max;
  d.wt = in->wt;
  d.rs = in->rs;
  d.nr = in->n_running;
  d.n = in->n_active;
  d.frozen_cmax = in->frozen_cmax;
  d.horizon = in->horizon;
  return d;
}

int resolve_cap(const ffs_instance *in, int32_t lds_slots) {
  int cap = lds_slots > 0 ? lds_slots : kDefaultLdsSlots;
  const int64_t h = align_up((size_t)in->horizon, 64);
  if (cap > h) cap = (int)h;
  cap = (int)align_up((size_t)(cap < 64 ? 64 : cap), 64);
  return cap;
}

size_t pq_bytes(const ffs_instance *in) {
  return align_up((size_t)in->n_jobs * in->n_stages * omp_of(in->o_max) * 4 + 64, 256);
}

size_t overflow_bytes(const ffs_instance *in, int32_t pop, int cap) {
  if (cap >= in->horizon) return 0;
  return align_up((size_t)pop * 4, 256) +
         (size_t)kFixBlocks * align_up((size_t)in->horizon + 64, 256);
}

struct DecodeLayout {
  Header *hdr;
  uint32_t *pq;
  int32_t *ovf_list;
  uint8_t *gprof;
  size_t gstride, total;
};

DecodeLayout decode_layout(void *ws, const ffs_instance *in, int32_t pop, int cap) {
  DecodeLayout L{};
  uint8_t *b = (uint8_t *)ws;
  size_t off = 0;
  L.hdr = (Header *)(b + off);
  off += kHeaderBytes;
  L.pq = (uint32_t *)(b + off);
  off += pq_bytes(in);
  if (cap < in->horizon) {
    L.ovf_list = (int32_t *)(b + off);
    off += align_up((size_t)pop * 4, 256);
    L.gstride = align_up((size_t)in->horizon + 64, 256);
    L.gprof = b + off;
    off += (size_t)kFixBlocks * L.gstride;
  }
  L.total = off;
  return L;
}

template <int MAXM>
int run_decode(const ffs_instance *in, const int32_t *prio, int32_t pop, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work, int cap, const DecodeLayout &L,
               hipStream_t stream) {
  const DInst d = make_dinst(in, L.pq);
  const size_t shmem = lds_bytes(in->n_active, cap);
  hipError_t e = launch(0, decode_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, prio, obj,
                        work, start, mach, L.hdr, L.ovf_list, cap);
  if (e != hipSuccess) return FFS_E_DEVICE;
  if (cap < in->horizon) {
    e = launch(3, overflow_kernel<MAXM>, dim3(kFixBlocks), dim3(kWave), lds_bytes(in->n_active, 0),
               stream, d, prio, obj, work, start, mach, L.hdr, (const int32_t *)L.ovf_list, L.gprof,
               L.gstride);
    if (e != hipSuccess) return FFS_E_DEVICE;
  }
  return FFS_OK;
}

int pack(const ffs_instance *in, uint32_t *pq, hipStream_t stream) {
  const int rows = in->n_jobs * in->n_stages;
  if (rows == 0) return FFS_OK;
  const int omp = omp_of(in->o_max);
  const int blocks = (int)((rows * (size_t)omp + 255) / 256);
  hipError_t e = launch(-1, pack_kernel, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, stream,
                        in->proc, in->power, pq, rows, in->o_max, omp);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

int read_header(Header *dev, Header *host, hipStream_t stream) {
  if (hipMemcpyAsync(host, dev, sizeof(Header), hipMemcpyDeviceToHost, stream) != hipSuccess)
    return FFS_E_DEVICE;
  if (hipStreamSynchronize(stream) != hipSuccess) return FFS_E_DEVICE;
  return FFS_OK;
}

int clear_header(Header *dev, hipStream_t stream) {
  return hipMemsetAsync(dev, 0, sizeof(Header), stream) == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

int err_code(int32_t err) {
  if (err & kErrInfeasible) return FFS_E_INFEASIBLE;
  if (err & kErrInval) return FFS_E_INVAL;
  return FFS_OK;
}

// GA workspace layout.
struct GaLayout {
  Header *hdr;
  uint32_t *pq;
  int32_t *prio[2];
  int64_t *obj[2];
  int32_t *elite;
  int64_t *elite_obj;
  int32_t *stage_prio;
  int64_t *stage_obj;
  int32_t *ovf_list;
  uint8_t *gprof;
  size_t gstride, total;
};

GaLayout ga_layout(void *ws, const ffs_instance *in, const ffs_ga_params *p, int cap) {
  GaLayout L{};
  uint8_t *b = (uint8_t *)ws;
  const size_t pop = (size_t)p->islands * p->rows * p->cols, n = (size_t)in->n_active;
  const size_t kk = p->mig_k > 0 ? p->mig_k : 1;
  size_t off = 0;
  L.hdr = (Header *)(b + off);
  off += kHeaderBytes;
  L.pq = (uint32_t *)(b + off);
  off += pq_bytes(in);
  for (int k = 0; k < 2; ++k) {
    L.prio[k] = (int32_t *)(b + off);
    off += align_up(pop * n * 4 + 4, 256);
    L.obj[k] = (int64_t *)(b + off);
    off += align_up(pop * 8, 256);
  }
  L.elite = (int32_t *)(b + off);
  off += align_up((size_t)p->islands * n * 4 + 4, 256);
  L.elite_obj = (int64_t *)(b + off);
  off += align_up((size_t)p->islands * 8, 256);
  L.stage_prio = (int32_t *)(b + off);
  off += align_up((size_t)p->islands * kk * n * 4 + 4, 256);
  L.stage_obj = (int64_t *)(b + off);
  off += align_up((size_t)p->islands * kk * 8, 256);
  L.ovf_list = (int32_t *)(b + off);
  off += align_up(pop * 4, 256);
  if (cap < in->horizon) {
    L.gstride = align_up((size_t)in->horizon + 64, 256);
    L.gprof = b + off;
    off += (size_t)kFixBlocks * L.gstride;
  }
  L.total = off;
  return L;
}

int check_ga_params(const ffs_ga_params *p) {
  if (!p || p->islands < 1 || p->rows < 1 || p->cols < 1 || p->mig_k < 0 || p->mig_interval < 0)
    return FFS_E_INVAL;
  const int64_t K = (int64_t)p->rows * p->cols;
  if (p->mig_k > K) return FFS_E_INVAL;
  if (K > 65536 || K * p->islands > (1 << 26)) return FFS_E_UNSUPPORTED;
  return FFS_OK;
}

GaDev make_gadev(const ffs_ga *ga, const GaLayout &L, int in_buf) {
  GaDev A;
  A.prio_in = L.prio[in_buf];
  A.obj_in = L.obj[in_buf];
  A.prio_out = L.prio[1 - in_buf];
  A.obj_out = L.obj[1 - in_buf];
  A.elite = L.elite;
  A.elite_obj = L.elite_obj;
  A.stage_prio = L.stage_prio;
  A.stage_obj = L.stage_obj;
  A.hdr = L.hdr;
  A.ovf_list = L.ovf_list;
  A.seed = ga->seed;
  A.shop = ga->shop;
  A.event = ga->event;
  A.rows = ga->params.rows;
  A.cols = ga->params.cols;
  A.islands = ga->params.islands;
  A.mig_k = ga->params.mig_k;
  A.pc = ga->params.pc;
  A.pm = ga->params.pm;
  return A;
}

template <int MAXM>
int ga_overflow(const ffs_instance *in, const GaLayout &L, int buf, int cap, hipStream_t stream) {
  if (cap >= in->horizon) return FFS_OK;
  const DInst d = make_dinst(in, L.pq);
  hipError_t e = launch(3, overflow_kernel<MAXM>, dim3(kFixBlocks), dim3(kWave),
                        lds_bytes(in->n_active, 0), stream, d, (const int32_t *)L.prio[buf],
                        L.obj[buf], (int64_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                        L.hdr, (const int32_t *)L.ovf_list, L.gprof, L.gstride);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

template <int MAXM>
int ga_init_impl(ffs_ga *ga, const ffs_instance *in, const GaLayout &L, hipStream_t stream) {
  const DInst d = make_dinst(in, L.pq);
  GaDev A = make_gadev(ga, L, 1);  // generation 0 is written to buffer 0
  const int pop = ga->pop, cap = ga->lds_slots, n = in->n_active;
  const int K = ga->params.rows * ga->params.cols;
  if (launch(1, ga_init_kernel<MAXM>, dim3(pop), dim3(kWave), lds_bytes(n, cap), stream, d, A,
             cap) != hipSuccess)
    return FFS_E_DEVICE;
  int rc = ga_overflow<MAXM>(in, L, 0, cap, stream);
  if (rc) return rc;
  if (launch(-1, elite_init_kernel, dim3(ga->params.islands), dim3(256), 0, stream,
             (const int32_t *)L.prio[0], (const int64_t *)L.obj[0], L.elite, L.elite_obj, K,
             n) != hipSuccess)
    return FFS_E_DEVICE;
  return FFS_OK;
}

template <int MAXM>
int ga_step_impl(ffs_ga *ga, const ffs_instance *in, int32_t n_gen, hipStream_t stream) {
  GaLayout L = ga_layout(ga->workspace, in, &ga->params, ga->lds_slots);
  const DInst d = make_dinst(in, L.pq);
  const int pop = ga->pop, cap = ga->lds_slots, n = in->n_active;
  const int K = ga->params.rows * ga->params.cols;
  const size_t shmem = lds_bytes(n, cap);
  for (int32_t k = 0; k < n_gen; ++k) {
    const int gen = ga->generation + 1;
    const int cur = ga->cur;
    GaDev A = make_gadev(ga, L, cur);
    if (launch(1, ga_generation_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, A, gen,
               cap) != hipSuccess)
      return FFS_E_DEVICE;
    int rc = ga_overflow<MAXM>(in, L, 1 - cur, cap, stream);
    if (rc) return rc;
    if (launch(2, replace_kernel, dim3(ga->params.islands), dim3(256), 0, stream, L.prio[1 - cur],
               L.obj[1 - cur], L.elite, L.elite_obj, K, n) != hipSuccess)
      return FFS_E_DEVICE;
    const ffs_ga_params &p = ga->params;
    if (p.mig_interval > 0 && p.mig_k > 0 && p.islands > 1 && gen % p.mig_interval == 0) {
      if (launch(-1, migrate_collect_kernel, dim3(p.islands), dim3(256), (size_t)K, stream,
                 (const int32_t *)L.prio[1 - cur], (const int64_t *)L.obj[1 - cur], L.stage_prio,
                 L.stage_obj, K, n, p.mig_k) != hipSuccess)
        return FFS_E_DEVICE;
      if (launch(-1, migrate_apply_kernel, dim3(p.islands), dim3(256), (size_t)K, stream,
                 L.prio[1 - cur], L.obj[1 - cur], L.elite, L.elite_obj,
                 (const int32_t *)L.stage_prio, (const int64_t *)L.stage_obj, K, n, p.mig_k,
                 p.islands) != hipSuccess)
        return FFS_E_DEVICE;
    }
    ga->cur = 1 - cur;
    ga->generation = gen;
  }
  return FFS_OK;
}

template <int MAXM>
void set_lds_limits() {
  static bool done = false;
  if (done) return;
  done = true;
  const int lim = max_lds_bytes();
  (void)hipFuncSetAttribute((const void *)decode_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)overflow_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)ga_generation_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)ga_init_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *ffs_strerror(int code) {
  switch (code) {
    case FFS_OK: return "ok";
    case FFS_E_INVAL: return "invalid argument or input";
    case FFS_E_INFEASIBLE: return "infeasible: an op needs more power than the peak limit";
    case FFS_E_WORKSPACE: return "workspace missing or too small";
    case FFS_E_DEVICE: return "HIP runtime error";
    case FFS_E_UNSUPPORTED: return "outside the limits of this build";
    default: return "unknown error";
  }
}

int ffs_prepare(ffs_instance *inst, void *workspace, size_t workspace_bytes, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (!workspace || workspace_bytes < FFS_PREPARE_WORKSPACE) return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Header *h = (Header *)workspace;
  if ((rc = clear_header(h, s))) return rc;
  PrepArgs a{inst->n_machines, inst->proc, inst->power, inst->first_stage, inst->ready,
             inst->machine_free, inst->running, inst->active, inst->n_jobs, inst->n_stages,
             inst->o_max, inst->q_max, inst->rs, inst->n_running, inst->n_active};
  if (launch(-1, prepare_kernel, dim3(1), dim3(1024), 0, s, a, h) != hipSuccess) return FFS_E_DEVICE;
  Header host;
  if ((rc = read_header(h, &host, s))) return rc;
  if ((rc = err_code(host.err))) return rc;
  if (host.horizon > INT_MAX / 2) return FFS_E_UNSUPPORTED;
  inst->horizon = (int32_t)host.horizon;
  return FFS_OK;
}

size_t ffs_decode_workspace_size(const ffs_instance *inst, int32_t pop, int32_t lds_slots) {
  if (check_host(inst) || inst->horizon < 1 || pop < 0) return 0;
  const int cap = resolve_cap(inst, lds_slots);
  return kHeaderBytes + pq_bytes(inst) + overflow_bytes(inst, pop, cap);
}

int ffs_decode(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots, void *workspace,
               size_t workspace_bytes, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (inst->horizon < 1 || pop < 0 || (pop > 0 && (!obj || (!prio && inst->n_active > 0))) ||
      ((start == nullptr) != (mach == nullptr)))
    return FFS_E_INVAL;
  if (pop == 0) return FFS_OK;
  const int cap = resolve_cap(inst, lds_slots);
  if (lds_bytes(inst->n_active, cap) > (size_t)max_lds_bytes()) return FFS_E_UNSUPPORTED;
  if (!workspace || workspace_bytes < ffs_decode_workspace_size(inst, pop, lds_slots))
    return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  DecodeLayout L = decode_layout(workspace, inst, pop, cap);
  if ((rc = clear_header(L.hdr, s))) return rc;
  if ((rc = pack(inst, L.pq, s))) return rc;
  if (inst->o_max <= 8) {
    set_lds_limits<8>();
    return run_decode<8>(inst, prio, pop, obj, start, mach, work, cap, L, s);
  }
  set_lds_limits<16>();
  return run_decode<16>(inst, prio, pop, obj, start, mach, work, cap, L, s);
}

int ffs_status(void *workspace, void *stream) {
  if (!workspace) return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Header host;
  int rc = read_header((Header *)workspace, &host, s);
  if (rc) return rc;
  const int32_t zero = 0;
  if (hipMemcpyAsync(&((Header *)workspace)->err, &zero, sizeof(zero), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFS_E_DEVICE;
  return err_code(host.err);
}

size_t ffs_ga_workspace_size(const ffs_instance *inst, const ffs_ga_params *params) {
  if (check_host(inst) || check_ga_params(params) || inst->horizon < 1) return 0;
  const int cap = resolve_cap(inst, params->lds_slots);
  return ga_layout(nullptr, inst, params, cap).total;
}

int ga_init(ffs_ga *ga, const ffs_instance *inst, const ffs_ga_params *params, uint64_t seed,
            uint64_t shop, int32_t event, void *workspace, size_t workspace_bytes, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (!ga || inst->horizon < 1) return FFS_E_INVAL;
  if ((rc = check_ga_params(params))) return rc;
  const int cap = resolve_cap(inst, params->lds_slots);
  if (lds_bytes(inst->n_active, cap) > (size_t)max_lds_bytes()) return FFS_E_UNSUPPORTED;
  const size_t need = ffs_ga_workspace_size(inst, params);
  if (!workspace || workspace_bytes < need) return FFS_E_WORKSPACE;
  memset(ga, 0, sizeof(*ga));
  ga->params = *params;
  ga->n_genes = inst->n_active;
  ga->pop = params->islands * params->rows * params->cols;
  ga->seed = seed;
  ga->shop = shop;
  ga->event = event;
  ga->generation = 0;
  ga->cur = 0;
  ga->workspace = workspace;
  ga->workspace_bytes = workspace_bytes;
  ga->lds_slots = cap;
  ga->n_jobs = inst->n_jobs;
  ga->horizon = inst->horizon;
  hipStream_t s = (hipStream_t)stream;
  GaLayout L = ga_layout(workspace, inst, params, cap);
  for (int k = 0; k < 2; ++k) {
    ga->prio[k] = L.prio[k];
    ga->obj[k] = L.obj[k];
  }
  ga->elite = L.elite;
  ga->elite_obj = L.elite_obj;
  if ((rc = clear_header(L.hdr, s))) return rc;
  if ((rc = pack(inst, L.pq, s))) return rc;
  if (inst->n_active == 0) {
    // No gene to decode: every individual is the empty vector with the frozen objective.
    std::vector<int64_t> o((size_t)ga->pop, (int64_t)inst->wt * inst->frozen_tardiness + inst->frozen_cmax);
    std::vector<int64_t> e((size_t)params->islands, o.empty() ? 0 : o[0]);
    if (hipMemcpyAsync(L.obj[0], o.data(), o.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(L.elite_obj, e.data(), e.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FFS_E_DEVICE;
    return FFS_OK;
  }
  if (inst->o_max <= 8) {
    set_lds_limits<8>();
    return ga_init_impl<8>(ga, inst, L, s);
  }
  set_lds_limits<16>();
  return ga_init_impl<16>(ga, inst, L, s);
}

int ga_step(ffs_ga *ga, const ffs_instance *inst, int32_t n_generations, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (!ga || !ga->workspace || n_generations < 0 || inst->n_active != ga->n_genes ||
      inst->n_jobs != ga->n_jobs || inst->horizon != ga->horizon)
    return FFS_E_INVAL;
  if (inst->n_active == 0) {
    ga->generation += n_generations;
    return FFS_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  if (inst->o_max <= 8) return ga_step_impl<8>(ga, inst, n_generations, s);
  return ga_step_impl<16>(ga, inst, n_generations, s);
}

int ga_view(const ffs_ga *ga, ffs_ga_view *view) {
  if (!ga || !view || !ga->workspace) return FFS_E_INVAL;
  view->prio = ga->prio[ga->cur];
  view->obj = ga->obj[ga->cur];
  view->elite = ga->elite;
  view->elite_obj = ga->elite_obj;
  view->work = (int64_t *)&((Header *)ga->workspace)->work;
  return FFS_OK;
}

int ga_best(const ffs_ga *ga, int32_t *prio_out, int64_t *obj_out, void *stream) {
  if (!ga || !ga->workspace || !obj_out || (ga->n_genes > 0 && !prio_out)) return FFS_E_INVAL;
  hipError_t e = launch(-1, best_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream,
                        (const int32_t *)ga->elite, (const int64_t *)ga->elite_obj,
                        ga->params.islands, ga->n_genes, prio_out, obj_out);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

size_t ffs_reschedule_workspace_size(int32_t n_jobs, int32_t n_new) {
  (void)n_jobs;
  (void)n_new;
  return kHeaderBytes;
}

int reschedule(const ffs_instance *prev, const int32_t *plan_start, const int32_t *plan_mach,
               int32_t rs, int32_t n_new, const int32_t *new_proc, const int32_t *new_power,
               const int32_t *new_release, const int32_t *new_due, ffs_instance *next,
               void *workspace, size_t workspace_bytes, void *stream) {
  int rc = check_host(prev);
  if (rc) return rc;
  if (!next || rs < prev->rs || n_new < 0 || (prev->n_jobs > 0 && (!plan_start || !plan_mach)) ||
      (n_new > 0 && (!new_proc || !new_power || !new_release || !new_due)) || !prev->release)
    return FFS_E_INVAL;
  if (prev->n_jobs + (int64_t)n_new >= (1 << 24)) return FFS_E_UNSUPPORTED;
  if (!next->proc || !next->power || !next->release || !next->due || !next->first_stage ||
      !next->ready || !next->machine_free || !next->running || !next->active)
    return FFS_E_INVAL;
  if (!workspace || workspace_bytes < ffs_reschedule_workspace_size(prev->n_jobs, n_new))
    return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Header *h = (Header *)workspace;
  if ((rc = clear_header(h, s))) return rc;
  ReschedArgs a{prev->n_machines, prev->proc, prev->power, prev->release, prev->due,
                prev->n_jobs, prev->n_stages, prev->o_max, prev->q_max, prev->rs,
                plan_start, plan_mach, rs, n_new, new_proc, new_power, new_release, new_due,
                (int32_t *)next->proc, (int32_t *)next->power, (int32_t *)next->release,
                (int32_t *)next->due, (int32_t *)next->first_stage, (int32_t *)next->ready,
                (int32_t *)next->machine_free, (int32_t *)next->running, (int32_t *)next->active,
                prev->n_stages * prev->o_max};
  if (launch(-1, reschedule_kernel, dim3(1), dim3(1024), 0, s, a, h) != hipSuccess)
    return FFS_E_DEVICE;
  Header host;
  if ((rc = read_header(h, &host, s))) return rc;
  if ((rc = err_code(host.err))) return rc;
  if (host.horizon > INT_MAX / 2) return FFS_E_UNSUPPORTED;
  next->n_jobs = prev->n_jobs + n_new;
  next->n_stages = prev->n_stages;
  next->o_max = prev->o_max;
  if (!next->n_machines) next->n_machines = prev->n_machines;
  next->q_max = prev->q_max;
  next->wt = prev->wt;
  next->rs = rs;
  next->n_running = host.n_running;
  next->frozen_tardiness = host.frozen_tardiness;
  next->frozen_cmax = host.frozen_cmax;
  next->n_active = host.n_active;
  next->horizon = (int32_t)host.horizon;
  return check_host(next);
}

int ffs_timing_enable(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (enable) {
    for (int f = 0; f < 4; ++f) {
      if (g_timing.ev[f].empty()) {
        g_timing.ev[f].resize(2 * kTimingPairs);
        for (auto &e : g_timing.ev[f])
          if (hipEventCreate(&e) != hipSuccess) return FFS_E_DEVICE;
      }
      g_timing.used[f] = 0;
      g_timing.ms[f] = 0;
      g_timing.launches[f] = 0;
    }
  }
  g_timing.on = enable != 0;
  return FFS_OK;
}

int ffs_timing_read(int32_t family, double *total_ms, int64_t *launches) {
  if (family < 0 || family > 3 || !total_ms || !launches) return FFS_E_INVAL;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (!g_timing.ev[family].empty()) {
    drain_family(family, g_timing.used[family]);
    g_timing.used[family] = 0;
  }
  *total_ms = g_timing.ms[family];
  *launches = g_timing.launches[family];
  return FFS_OK;
}

}  // extern "C"
