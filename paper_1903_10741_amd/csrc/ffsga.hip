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

#include <atomic>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ffs_surrogate.h"
#include "ffsga.h"

typedef unsigned long long u64;
typedef __attribute__((address_space(4))) const int32_t c_i32;
typedef __attribute__((address_space(4))) const uint32_t c_u32;
typedef __attribute__((address_space(4))) const int64_t c_i64;

// Workspace of ffs_decode_noalloc: one copy per GPU, held until the process
// ends, shared by every such call on that GPU.
static __device__ __align__(256) uint8_t scratch[FFS_DECODE_SCRATCH_BYTES];

namespace {

constexpr int kWave = 64;
constexpr int kMaxGenes = 4096;
constexpr int kMaxStages = 127;
constexpr int kDefaultLdsSlots = 4096;
constexpr int kFixBlocks = 64;       // overflow decodes in flight at once
constexpr int kHeaderBytes = 256;
constexpr int kMaxTime = 1 << 27;    // completion times pack as (time << 4 | machine)
// Free time of the lanes that hold no machine of the stage: their machine key
// (kNoMachine + p) << 4 | lane stays above every real key and below 2^32.
constexpr int kNoMachine = 0x0FFF0000;
static_assert(kNoMachine >= kMaxTime && kNoMachine + 0xFFFF < (1 << 28), "machine key");

// Device-side status word and small results at the head of every workspace.
struct Header {
  int32_t err;          // bit 0: invalid input, bit 1: infeasible power
  int32_t ovf_count;    // decodes waiting for the overflow kernel
  int32_t ovf_done;     // overflow blocks finished (last one resets)
  int32_t pad0;
  int64_t horizon;
  int64_t frozen_tardiness;
  int32_t frozen_cmax, n_running, n_active, n_ops;  // n_ops: unfrozen ops (ffs_prepare)
  unsigned long long work;  // algorithmic work of every decode of a GA
  int32_t span_max;     // longest schedule (end - RS) of a sizing decode (FFS_LDS_AUTO)
  int32_t n_fixed;      // planned ops kept in place (reschedule_static)
  int64_t e_max;        // eq. (13)'s E_max of a classical GA (FFS_GA_CLASSICAL)
  unsigned long long overflows;  // decodes of a GA that outgrew the on-chip profile
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

// v_writelane: a uniform value into one lane of a register (bound to the LLVM
// intrinsic by name; hipcc has no builtin for it).
extern "C" __device__ int ffs_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
__device__ __forceinline__ u64 readlane64(u64 v, int lane) {
  return (u64)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane) << 32 |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
// A wave-uniform unsigned sum read out to the scalar side.
__device__ __forceinline__ u64 uniform_sum(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ u64 uniform_sum(u64 v) { return readlane64(v, 0); }

// Lane mask of a predicate across the wave.
__device__ __forceinline__ u64 ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// ---------------------------------------------------------------------------
// Instance as the kernels see it.
// ---------------------------------------------------------------------------
struct DInst {
  const uint32_t *pq;        // [n][g][omp]: P | Q << 16 of the active jobs, in gene order
  const int32_t *due_k;      // [n]: due dates of the active jobs, in gene order
  const int32_t *nm;         // [g]
  const int32_t *due;        // [n_jobs]
  const int32_t *first;      // [n_jobs]
  const int32_t *ready;      // [n_jobs]
  const int32_t *mfree;      // [g][om]
  const int32_t *running;    // [nr][2]
  const int32_t *active;     // [n]
  const int32_t *fixed;      // [nf][3]: (start, end, q) of planned ops kept in place
  int64_t frozen_t;
  int32_t n_jobs, g, om, omp, q_max, wt, rs, nr, n, frozen_cmax, horizon, nf;
  int32_t rules;  // FFS_RULE_* decode variants (job-priority chromosomes)
};

template <class T>
__device__ __forceinline__ T ld_const(const T *p, size_t i) {
  typedef __attribute__((address_space(4))) const T cT;
  return ((cT *)p)[i];
}

// Profile with one byte per slot in LDS.
struct LdsProfile {
  // a commit adds each slot's byte from its own lane (the LDS serialises the
  // four adds to one word), with no sum across a quad first
  static constexpr bool kLaneAdds = true;
  uint8_t *p;
  int cap;
  __device__ void clear() const {
    uint32_t *w = (uint32_t *)p;
    for (int x = __lane_id(); x < (cap + kWave) / 4; x += kWave) w[x] = 0;
  }
  __device__ uint32_t get(int x) const { return p[x]; }
  __device__ void add(int x, uint32_t q) const {
    atomicAdd((uint32_t *)(p + (x & ~3)), q << (8 * (x & 3)));
  }
  // Add four packed byte increments to the word of slots [x4, x4 + 4), x4 % 4 == 0.
  __device__ void add_word(int x4, uint32_t w) const { atomicAdd((uint32_t *)(p + x4), w); }
  __device__ void order() const { __asm__ volatile("" ::: "memory"); }
  __device__ int place(int t0, int p, uint32_t thr) const;
  __device__ void commit(int t, int p, int q) const;
  __device__ void add_running(int len, int q) const {
    for (int x = __lane_id(); x < len; x += kWave) add(x, (uint32_t)q);
  }
  __device__ void add_span(int a, int b, int q) const {
    for (int x = a + __lane_id(); x < b; x += kWave) add(x, (uint32_t)q);
  }
};

// Slots of an off-chip profile: the horizon bound rounded up to a multiple of
// 64, like every on-chip cap, so that the commit's clamp onto the last word
// stays word-aligned and only ever absorbs slots no finished decode reaches.
// Its region holds offchip_cap + 64 bytes (the zero slots after it).
__host__ __device__ inline int offchip_cap(int horizon) {
  return (int)align_up((size_t)horizon, 64);
}

// Profile with one byte per slot in global memory (overflow tier). Each
// profile belongs to one single-wave block, so work-group scope orders the
// lanes' updates and reads; nothing else touches it.
struct GlobalProfile {
  // a commit sums each quad's bytes first and adds one word per quad (global
  // atomics to one word from several lanes would queue at the cache)
  static constexpr bool kLaneAdds = false;
  uint8_t *p;
  int cap;
  __device__ void clear() const {
    uint32_t *w = (uint32_t *)p;
    for (int x = __lane_id(); x < (cap + kWave) / 4; x += kWave)
      __hip_atomic_store(w + x, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    order();
  }
  __device__ uint32_t get(int x) const {
    uint32_t w = __hip_atomic_load((uint32_t *)(p + (x & ~3)), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    return (w >> (8 * (x & 3))) & 0xFFu;
  }
  __device__ void add(int x, uint32_t q) const {
    __hip_atomic_fetch_add((uint32_t *)(p + (x & ~3)), q << (8 * (x & 3)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ void add_word(int x4, uint32_t w) const {
    __hip_atomic_fetch_add((uint32_t *)(p + x4), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ void order() const { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup"); }
  __device__ int place(int t0, int p, uint32_t thr) const;
  __device__ void commit(int t, int p, int q) const;
  __device__ void add_running(int len, int q) const {
    for (int x = __lane_id(); x < len; x += kWave) add(x, (uint32_t)q);
  }
  __device__ void add_span(int a, int b, int q) const {
    for (int x = a + __lane_id(); x < b; x += kWave) add(x, (uint32_t)q);
  }
};

// Push right (Algorithm 2) over a byte profile: the earliest t >= t0 with
// every slot of [t, t + p) at most thr. The lanes hold the 64 slots
// [scan, scan + 64); a ballot marks the window's slots that break the peak and
// t jumps past the last of them, re-testing the same chunk; a clean window
// part that runs off the chunk moves on to the next 64 slots. Reads past cap
// land in the 64 zero slots after it. The re-tests form an inner loop and the
// branches carry the common case's odds (no slot breaks the peak, the window
// ends in the first chunk), so that case runs straight through.
template <class Prof>
__device__ __forceinline__ int place_bytes(const Prof &prof, int t0, int p, uint32_t thr) {
  const int lane = __lane_id(), cap = prof.cap;
  int t = t0, top = min(t0, cap) + kWave;  // the chunk is [top - 64, top)
  int sl = top - kWave + lane;              // this lane's slot
  uint32_t v = prof.get(sl);
  for (;;) {
    // slots of [t, t + p) in this chunk (one unsigned compare) that break the peak
    u64 hit = ballot64((uint32_t)(sl - t) < (uint32_t)p) & ballot64(v > thr);
    while (__builtin_expect(hit != 0, 0)) {
      t = top - (int)__clzll(hit);
      hit = ballot64((uint32_t)(sl - t) < (uint32_t)p) & ballot64(v > thr);
    }
    if (__builtin_expect(t + p <= top || top >= cap, 1)) break;
    top += kWave;
    sl += kWave;
    v = prof.get(sl);
  }
  return t;
}

// Commit q on [t, t + p) of a byte profile. The lanes cover the word-aligned
// slots [base, base + 64), lane i slot base + i. Bytes never carry into each
// other (every byte stays <= Q_max), so a word may take its four slots'
// increments as four adds or as one: on chip each lane of the window adds its
// own byte; off chip each quad of lanes sums its bytes across the quad and its
// first lane adds the word (quads outside the window add zero: cheaper than
// testing for it). Slots past cap (the decode is then redone off chip) are
// clamped onto the last word, so the zero slots after cap stay zero.
//
// In two halves: commit_word forms the increments (registers only), commit_add
// adds them; an op loop can place independent work between the two.
template <class Prof>
__device__ __forceinline__ uint32_t commit_word(int t, int p, int q) {
  const int lane = __lane_id();
  if (Prof::kLaneAdds) return (uint32_t)q << (8 * (lane & 3));  // commit_add masks the window
  const int base = t & ~3;
  uint32_t c = (uint32_t)(base + lane - t) < (uint32_t)p ? (uint32_t)q << (8 * (lane & 3)) : 0u;
  c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0xB1, 0xF, 0xF, false);
  c += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)c, 0x4E, 0xF, 0xF, false);
  return c;
}
template <class Prof>
__device__ __forceinline__ void commit_add(const Prof &prof, int t, int p, int q, uint32_t c) {
  const int lane = __lane_id(), cap = prof.cap;
  const int base = t & ~3;
  if (Prof::kLaneAdds) {
    if ((uint32_t)(base + lane - t) < (uint32_t)p) prof.add_word(min(base + (lane & ~3), cap - 4), c);
  } else if ((lane & 3) == 0) {
    prof.add_word(min(base + lane, cap - 4), c);
  }
  if (__builtin_expect(t - base + p > kWave, 0))  // windows longer than the lanes
    for (int b = base + kWave + lane; b < t + p; b += kWave) prof.add(min(b, cap - 1), (uint32_t)q);
  prof.order();
}
template <class Prof>
__device__ __forceinline__ void commit_bytes(const Prof &prof, int t, int p, int q) {
  commit_add(prof, t, p, q, commit_word<Prof>(t, p, q));
}

__device__ __forceinline__ int LdsProfile::place(int t0, int p, uint32_t thr) const {
  return place_bytes(*this, t0, p, thr);
}
__device__ __forceinline__ void LdsProfile::commit(int t, int p, int q) const {
  commit_bytes(*this, t, p, q);
}
__device__ __forceinline__ int GlobalProfile::place(int t0, int p, uint32_t thr) const {
  return place_bytes(*this, t0, p, thr);
}
__device__ __forceinline__ void GlobalProfile::commit(int t, int p, int q) const {
  commit_bytes(*this, t, p, q);
}

enum : int { kDecOk = 0, kDecOverflow = 1, kDecInval = 2, kDecInfeasible = 3 };

// LDS of one wave (one chromosome of n genes; words of a packed P|Q row per op):
//   rdy   [n+1]      by rank: completion of the job's last placed stage, slots after RS
//                    (scratch before the decode); an op's end replaces it as soon as the
//                    op is placed
//   jobs  [n+2]      by rank: 16-bit gene index | min(first_stage, 15) << 12
//                    (correction scratch before the decode)
//   op    [n+2]      the current stage's ops in order, as 16-bit ranks (two spare
//                    records that the op loop prefetches past the last)
//   rec   [kRing]    packed P | Q << 16 rows of the stage's ops, one word per machine,
//                    staged from the packed table kWave / o_s ops at a time
//   prof  [cap+64]   power in use per time slot after RS, one byte per slot (the last
//                    64 stay zero so a chunk read never needs clamping)
//   gene  [n]        the chromosome (input), at the start of prof's region (which holds
//                    at least n words): it is dead once the decode has built the ranks,
//                    before the profile is cleared
//
// The hybrid GA's generation and init kernels, under the default decode rules,
// use a narrow form of the same layout (`LdsN`): rdy in 16 bits, clamped to
// [0, 65535] when loaded ([n+2] halfwords at the start, then jobs and op). A
// time of 65535 or more exceeds every on-chip profile (at most 32 768 slots), so
// such a decode overflows anyway, and an op's end is read only at the job's next
// stage, after the stage's overflow check; 0 for a job ready before RS changes
// no start (every use takes a max with a machine's free time, at least 0). A
// decode redone off chip lays the wide form over the same allocation.
template <class R>
struct LdsT {
  int32_t *gene;
  R *rdy;
  uint16_t *jobs, *op;
  uint32_t *rec;
  uint8_t *prof;
};
using Lds = LdsT<int32_t>;
using LdsN = LdsT<uint16_t>;

// Breeding scratch inside a decode's LDS (free until the decode builds its
// ranks): n + 1 words and n halfwords.
__device__ __forceinline__ int32_t *scratch32(const Lds &l) { return l.rdy; }
__device__ __forceinline__ uint16_t *scratch16(const Lds &l) { return l.jobs; }
__device__ __forceinline__ int32_t *scratch32(const LdsN &l) { return (int32_t *)l.jobs; }
__device__ __forceinline__ uint16_t *scratch16(const LdsN &l) { return l.rdy; }

// Words of one row-ring buffer: a chunk of kWave / o_s ops of o_s words each,
// plus the record the op loop prefetches one past the chunk (read, never used).
constexpr int kRing = kWave + 16;

// LDS bytes before the profile region, and in all (cap = 0: no on-chip profile,
// the region still holds the genes).
__host__ __device__ inline size_t lds_head(int n) {
  return align_up((size_t)4 * n + 4, 16) + 2 * align_up((size_t)2 * n + 4, 16) + 4 * kRing;
}
__host__ __device__ inline size_t lds_bytes(int n, int cap) {
  const size_t prof = cap > 0 ? align_up(cap, 16) + kWave : 0, gene = align_up((size_t)4 * n, 16);
  return lds_head(n) + (prof > gene ? prof : gene);
}
// The narrow form (LdsN), with room for the wide form of an off-chip redo.
__host__ __device__ inline size_t lds_head_n(int n) {
  return 3 * align_up((size_t)2 * n + 4, 16) + 4 * kRing;
}
__host__ __device__ inline size_t lds_bytes_n(int n, int cap) {
  const size_t prof = cap > 0 ? align_up(cap, 16) + kWave : 0, gene = align_up((size_t)4 * n, 16);
  const size_t narrow = lds_head_n(n) + (prof > gene ? prof : gene), redo = lds_head(n) + gene;
  return narrow > redo ? narrow : redo;
}

__device__ __forceinline__ Lds carve_lds(uint8_t *smem, int n) {
  Lds l;
  const size_t a = align_up((size_t)4 * n + 4, 16), b = align_up((size_t)2 * n + 4, 16);
  l.rdy = (int32_t *)smem;
  l.jobs = (uint16_t *)(smem + a);
  l.op = (uint16_t *)(smem + a + b);
  l.rec = (uint32_t *)(smem + a + 2 * b);
  l.prof = (uint8_t *)l.rec + 4 * kRing;
  l.gene = (int32_t *)l.prof;
  return l;
}
__device__ __forceinline__ LdsN carve_lds_n(uint8_t *smem, int n) {
  LdsN l;
  const size_t b = align_up((size_t)2 * n + 4, 16);
  l.rdy = (uint16_t *)smem;
  l.jobs = (uint16_t *)(smem + b);
  l.op = (uint16_t *)(smem + 2 * b);
  l.rec = (uint32_t *)(smem + 3 * b);
  l.prof = (uint8_t *)l.rec + 4 * kRing;
  l.gene = (int32_t *)l.prof;
  return l;
}

// Minimum over lanes 0..MAXM-1 of v, left in lane MAXM-1 (DPP quad permutes,
// then row shifts; lanes outside the row contribute the identity).
template <int MAXM>
__device__ __forceinline__ uint32_t machine_min(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0xB1, 0xF, 0xF, false));
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x4E, 0xF, 0xF, false));
  if (MAXM > 4)
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x114, 0xF, 0xF, false));
  if (MAXM > 8)
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x118, 0xF, 0xF, false));
  return v;
}

// The same minimum as a scalar: up to 4 machines one readlane of the quad
// minimum; 8 the smaller of two quads' minima read out (two readlanes and a
// scalar min instead of a third DPP step and its wait states).
template <int MAXM>
__device__ __forceinline__ uint32_t machine_min_scalar(uint32_t v) {
  if (MAXM == 8) {
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0xB1, 0xF, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)v, 0x4E, 0xF, 0xF, false));
    return min((uint32_t)__builtin_amdgcn_readlane((int)v, 3),
               (uint32_t)__builtin_amdgcn_readlane((int)v, 7));
  }
  return (uint32_t)__builtin_amdgcn_readlane((int)machine_min<MAXM>(v), MAXM - 1);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ int wave_max32(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  return v;
}

// Whether the job of packed rank record jk has an op at stage s: its first
// unfrozen stage is at most s. The record holds min(first stage, 15), exact
// unless the stage is 15 or later with more than 16 stages (`exact`, uniform:
// then a record of 15 is looked up).
__device__ __forceinline__ bool live_at(const DInst &I, uint32_t jk, int s, bool exact) {
  bool live = (int)(jk >> 12) <= s;
  if (exact && (jk >> 12) == 15) live = ld_const(I.first, ld_const(I.active, jk & 0xFFF)) <= s;
  return live;
}

// Decode the chromosome in l.gene (Section 4.3, Algorithm 2, eq. (1)) with the
// power profile `prof`. On kDecOk lane 0 has written *obj_out. Every lane
// calls this; the result is uniform.
//
// Per stage, the lanes first gather the stage's ops in decode order (jobs by
// decreasing priority whose first unfrozen stage is reached) with their
// earliest start and packed P|Q row. Then each op runs on the whole wave:
// lane m computes the completion on machine m (its free time lives in lane m)
// and a DPP minimum over (completion << 4 | m) picks the machine of earliest
// completion, lowest index on ties; the push-right reads 64 profile slots at
// once and a ballot marks those that would break the peak; the scalar unit
// moves the start past the last of them inside the window.
//
// RULES: false compiles the default rules only (no per-op rule test);
// true reads I.rules (FFS_RULE_*). decode_core picks once per decode.
template <int MAXM, bool PLAN, bool RULES, class L, class Prof>
__device__ int decode_core_rules(const DInst &I, const L &l, Prof &&prof, int64_t *obj_out,
                                 int64_t *work_out, int32_t *start_out, int32_t *mach_out,
                                 int32_t *span_max) {
  using R = typename std::remove_pointer<decltype(l.rdy)>::type;
  constexpr bool kNarrow = std::is_same<R, uint16_t>::value;
  static_assert(!kNarrow || (!PLAN && !RULES), "narrow layout: default rules, no plan");
  const int lane = __lane_id();
  const int n = I.n;
  const u64 below = (1ull << lane) - 1;
  // Rank of gene k: n - prio_k (larger priority first). Times from here on
  // count slots after RS (a job ready before RS has a negative ready time).
  const int rs = I.rs;
  for (int x = lane; x < n; x += kWave) l.jobs[x] = 0xFFFF;
  int bad = 0;
  __asm__ volatile("" ::: "memory");
  for (int k = lane; k < n; k += kWave) {
    const int v = l.gene[k];
    if (v >= 1 && v <= n) l.jobs[n - v] = (uint16_t)k;
    else bad = 1;
  }
  __asm__ volatile("" ::: "memory");
  for (int x = lane; x < n; x += kWave) {
    const int k = l.jobs[x];
    if (k == 0xFFFF) {
      bad = 1;
    } else {
      const int j = ld_const(I.active, k);
      l.jobs[x] = (uint16_t)(k | min(ld_const(I.first, j), 15) << 12);
      // may be negative: every use takes a max with a machine's free time, at least 0
      const int r = ld_const(I.ready, j) - rs;
      l.rdy[x] = kNarrow ? (R)min(max(r, 0), 0xFFFF) : (R)r;
    }
  }
  if (ballot64(bad)) return kDecInval;

  // Power held by the ops running at RS, on [RS, end), and by the planned ops
  // kept in place (the static approach), on their own windows.
  prof.clear();
  prof.order();
  for (int r = 0; r < I.nr; ++r) {
    const int len = ld_const(I.running, 2 * r) - I.rs;
    const uint32_t q = (uint32_t)ld_const(I.running, 2 * r + 1);
    if (len > prof.cap) return kDecOverflow;
    prof.add_running(len, (int)q);
  }
  for (int r = 0; r < I.nf; ++r) {
    const int b = ld_const(I.fixed, 3 * r + 1) - I.rs;
    if (b > prof.cap) return kDecOverflow;
    prof.add_span(ld_const(I.fixed, 3 * r) - I.rs, b, ld_const(I.fixed, 3 * r + 2));
  }
  prof.order();

  const int cap = prof.cap;
  const bool power_ect = RULES && (I.rules & FFS_RULE_POWER_ECT) != 0;
  const bool fifo = RULES && (I.rules & FFS_RULE_FIFO) != 0;
  int64_t work = 0;
  for (int s = 0; s < I.g; ++s) {
    const int os = ld_const(I.nm, s);
    int fr = lane < os ? max(ld_const(I.mfree, (size_t)s * I.om + lane) - rs, 0) : kNoMachine;
    // The stage's ops, compacted in decode order (by rank, i.e. priority, or
    // with FFS_RULE_FIFO by the completion of the previous stage, then rank),
    // plus a spare record so the op loop can prefetch one past the last.
    int cnt = 0;
    // FFS_RULE_FIFO with at most 128 jobs: keys (completion << 32 | rank) of the
    // stage's jobs in two registers, all ones for jobs not at this stage; a
    // job's place is the number of keys below its own, counted against keys
    // broadcast one lane at a time.
    const bool fifo_reg = fifo && n <= 2 * kWave;
    const bool exact = I.g > 16 && s >= 15;
    u64 fk0 = ~0ull, fk1 = ~0ull;
    if (fifo_reg) {
      if (lane < n && live_at(I, l.jobs[lane], s, exact))
        fk0 = (u64)(uint32_t)(l.rdy[lane] + rs) << 32 | (uint32_t)lane;
      if (kWave + lane < n && live_at(I, l.jobs[kWave + lane], s, exact))
        fk1 = (u64)(uint32_t)(l.rdy[kWave + lane] + rs) << 32 | (uint32_t)(kWave + lane);
    }
    for (int b = 0; b < n; b += kWave) {
      const int x = b + lane;
      const bool live = x < n && live_at(I, l.jobs[x], s, exact);
      const u64 mk = ballot64(live);
      if (live) {
        int k = cnt + __popcll(mk & below);
        if (fifo_reg) {
          const u64 kx = b == 0 ? fk0 : fk1;
          k = 0;
          for (int y = 0; y < min(n, kWave); ++y)
            k += readlane64(fk0, y) < kx;
          for (int y = kWave; y < n; ++y)
            k += readlane64(fk1, y - kWave) < kx;
        } else if (fifo) {
          const int cx = l.rdy[x];
          k = 0;
          for (int y = 0; y < n; ++y) {
            const int cy = l.rdy[y];
            k += live_at(I, l.jobs[y], s, exact) && (cy < cx || (cy == cx && y < x));
          }
        }
        l.op[k] = (uint16_t)x;
      }
      cnt += __popcll(mk);
    }
    if (lane < 2) l.op[cnt + lane] = 0;
    __asm__ volatile("" ::: "memory");
    // The ops' packed P|Q rows come from the packed table chunk by chunk: lane
    // lk * o_s + lm holds machine lm of op lk of a chunk of kWave / o_s ops.
    // The rows of chunk c + 1 are loaded while chunk c runs and stored over
    // chunk c's when it ends (after its last read: LDS keeps a wave's order),
    // so the loads' latency stays hidden and LDS holds one chunk instead of the
    // whole stage.
    const int C = kWave / os, lk = lane / os, lm = lane - lk * os;
    const uint32_t *pq_stage = I.pq + (size_t)s * I.omp + lm;
    const size_t pq_job = (size_t)I.g * I.omp;
    auto row_word = [&](int k) -> uint32_t {
      if (lk >= C || k >= cnt) return 0u;
      return pq_stage[(size_t)(l.jobs[l.op[k]] & 0xFFF) * pq_job];
    };
    {
      const uint32_t w0 = row_word(lk);
      if (lk < C) l.rec[lane] = w0;
    }
    __asm__ volatile("" ::: "memory");
    // The record pointer as a per-lane value (the asm hides that the zero is
    // uniform): records are then read through one vector address with immediate
    // offsets instead of a scalar address moved in every op. The op loop reads
    // the rank of the op after next and the ready time of the next op's job
    // (the completion of its previous stage, still in rdy: each job has one op
    // per stage) one op ahead, and writes each op's end into rdy at once.
    int vz;
    __asm__("v_mov_b32 %0, 0" : "=v"(vz));
    const uint16_t *opp = l.op + vz;
    R *rdy_at = l.rdy + opp[0];  // the current op's job
    int rk1 = opp[1];                  // the next op's rank
    int ex = *rdy_at;                  // the current op's job's ready time
    // The stage's work sum, per lane (summed on the vector unit). Default rules:
    // the push-right intervals [t0, t) of one machine's ops are disjoint and lie
    // within the span after RS (< 2^27 slots), so over at most 16 machines they
    // add up to at most 2^31, and the 2p terms to at most 2 * 4096 * 65535 < 2^29:
    // unsigned 32 bits hold the sum. The power-aware rule pushes several machines
    // right per op, over the same slots again for later ops: 64 bits.
    using StageWork = typename std::conditional<RULES, u64, uint32_t>::type;
    StageWork stage_work = (StageWork)(uint32_t)vz;
    // Each op's profile update is issued by the next op, after its machine choice
    // and before its first profile read: the update's vector work then fills the
    // machine choice's dependency gaps instead of lengthening the op's chain. The
    // stage's first op updates an empty window (p = 0 adds nothing).
    int ct = 0, cp = 0, cq = 0;
    for (int base = 0; base < cnt; base += C) {
      const uint32_t next_w = row_word(base + C + lk);  // in flight during this chunk
      const uint32_t *recp = l.rec + min(lane, os - 1);
      uint32_t pqv = *recp;
      // Every LDS read before the op loop has landed (lgkmcnt 0): the wait sits
      // here, and the loop's head, which this read and the op loop's own reads
      // reach, does not wait for the previous op's profile and end stores.
      __builtin_amdgcn_s_waitcnt(0xC07F);
      const int k_end = min(base + C, cnt);
    for (int k = base; k < k_end; ++k) {
      opp += 1;
      recp += os;
      const int rk2 = opp[1];
      R *const rdy_next = l.rdy + rk1;
      const int ex_next = *rdy_next;
      const uint32_t pq_next = *recp;
      // the previous op's profile words, formed while this op's keys reduce
      const uint32_t cword = commit_word<typename std::decay<decltype(prof)>::type>(ct, cp, cq);
      // Machine of earliest completion (ties to the lowest index).
      const int t0v = max(ex, fr);  // earliest start on this lane's machine
      const uint32_t key = ((uint32_t)(t0v + (int)(pqv & 0xFFFFu)) << 4) | (uint32_t)lane;
      uint32_t kmin = machine_min_scalar<MAXM>(key);
      int t = 0;
      StageWork cw = 0;
      if (power_ect) {
        prof.commit(ct, cp, cq);  // the previous op of the stage
        // FFS_RULE_POWER_ECT: the earliest completion after the machine's push-right
        // (ties to the lowest index). The key above, (completion ignoring power) << 4
        // | machine, bounds a machine's key after its push-right from below: the
        // machine of least key goes first, then in index order only machines whose
        // key is below the best so far. Work: 3 per machine, plus the examined
        // slots and p of every machine pushed right.
        const int ox = uni(ex);  // uniform: keeps this loop on the scalar unit
        const int first = (int)(kmin & 15u);
        uint32_t best = 0xFFFFFFFFu;
        cw = 3 * os;
        for (int k = -1; k < os; ++k) {
          const int m = k < 0 ? first : k;
          if (k >= 0 && m == first) continue;
          if ((uint32_t)__builtin_amdgcn_readlane((int)key, m) >= best) continue;
          const uint32_t pqm = (uint32_t)__builtin_amdgcn_readlane((int)pqv, m);
          const int pm = (int)(pqm & 0xFFFFu);
          const int t0m = max(ox, __builtin_amdgcn_readlane(fr, m));
          const int tm = prof.place(t0m, pm, (uint32_t)(I.q_max - (int)(pqm >> 16)));
          cw += (StageWork)((tm - t0m) + pm);
          const uint32_t km = ((uint32_t)(tm + pm) << 4) | (uint32_t)m;
          if (km < best) {
            best = km;
            t = tm;
          }
        }
        kmin = best;
      }
      const int mb = (int)(kmin & 15u);
      const uint32_t pq = (uint32_t)__builtin_amdgcn_readlane((int)pqv, mb);
      const int p = (int)(pq & 0xFFFFu), q = (int)(pq >> 16);
      if (!power_ect) {
        // Q > Q_max is rejected by the instance checks; even then the unsigned
        // threshold only makes every slot pass, so the push-right still ends.
        const int t0 = __builtin_amdgcn_readlane(t0v, mb);
        commit_add(prof, ct, cp, cq, cword);  // the previous op of the stage
        t = prof.place(t0, p, (uint32_t)(I.q_max - q));
        cw = (StageWork)((t - t0) + 2 * p);
      } else {
        cw += (StageWork)p;
      }
      ct = t;
      cp = p;
      cq = q;
      const int end = t + p;
      fr = ffs_writelane(end, mb, fr);
      *rdy_at = (R)(PLAN ? end | (mb << 27) : end);
      stage_work = stage_work + cw;
      rdy_at = rdy_next;
      rk1 = rk2;
      ex = ex_next;
      pqv = pq_next;
    }
      if (lk < C) l.rec[lane] = next_w;
      __asm__ volatile("" ::: "memory");
    }
    prof.commit(ct, cp, cq);  // the stage's last op
    work += (int64_t)uniform_sum(stage_work) + (power_ect ? 0 : 3 * os * cnt);
    if (wave_max32(lane < os ? fr : 0) > cap) return kDecOverflow;
    __asm__ volatile("" ::: "memory");
    // With a plan: start and machine of every op, and the machine bits taken
    // out of the jobs' completion times.
    if (PLAN) {
      for (int k = lane; k < cnt; k += kWave) {
        const int x = l.op[k];
        const int e = l.rdy[x];
        const int end = e & (kMaxTime - 1), mb = e >> 27;
        const size_t gk = l.jobs[x] & 0xFFF, j = (size_t)ld_const(I.active, gk);
        l.rdy[x] = end;
        const uint32_t pqb = I.pq[(gk * I.g + s) * I.omp + mb];
        start_out[j * I.g + s] = end + rs - (int)(pqb & 0xFFFFu);
        mach_out[j * I.g + s] = mb;
      }
      __asm__ volatile("" ::: "memory");
    }
  }
  // Objective, eqs. (1)-(3), over every job in J u J'.
  int64_t tard = 0;
  int cmax = 0;
  for (int x = lane; x < n; x += kWave) {
    const int c = (int)l.rdy[x] + rs;
    const int late = c - ld_const(I.due_k, l.jobs[x] & 0xFFF);
    tard += late > 0 ? late : 0;
    cmax = max(cmax, c);
  }
  tard = wave_sum64(tard);
  cmax = wave_max32(cmax);
  if (span_max && lane == 0) atomicMax(span_max, cmax - rs);  // profile slots this decode used
  cmax = max(cmax, I.frozen_cmax);
  if (lane == 0) {
    *obj_out = (int64_t)I.wt * (I.frozen_t + tard) + cmax;
    if (work_out) *work_out = work;
  }
  return kDecOk;
}

template <int MAXM, bool PLAN, class Prof>
__device__ __forceinline__ int decode_core(const DInst &I, const Lds &l, Prof &&prof,
                                           int64_t *obj_out, int64_t *work_out,
                                           int32_t *start_out, int32_t *mach_out,
                                           int32_t *span_max = nullptr) {
  if (I.rules == 0)
    return decode_core_rules<MAXM, PLAN, false>(I, l, prof, obj_out, work_out, start_out, mach_out,
                                                span_max);
  return decode_core_rules<MAXM, PLAN, true>(I, l, prof, obj_out, work_out, start_out, mach_out,
                                             span_max);
}
// The narrow layout serves the default rules only (its callers check I.rules).
template <int MAXM, bool PLAN, class Prof>
__device__ __forceinline__ int decode_core(const DInst &I, const LdsN &l, Prof &&prof,
                                           int64_t *obj_out, int64_t *work_out,
                                           int32_t *start_out, int32_t *mach_out,
                                           int32_t *span_max = nullptr) {
  return decode_core_rules<MAXM, false, false>(I, l, prof, obj_out, work_out, start_out, mach_out,
                                               span_max);
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
  const LdsProfile prof{l.prof, cap};
  int64_t *w = work ? work + i : nullptr;
  const int st = start ? decode_core<MAXM, true>(I, l, prof, obj + i, w, start + plan, mach + plan)
                       : decode_core<MAXM, false>(I, l, prof, obj + i, w, nullptr, nullptr);
  if (st == kDecOk) return;
  if (__lane_id() == 0) obj[i] = -1;
  if (st == kDecOverflow) push_overflow(hdr, ovf_list, i);
  else flag_error(hdr, st);
}

// Redo the decodes listed as overflowed with a global-memory profile of
// `horizon` slots per block; the last block to finish clears the list. span:
// null, or where the longest schedule is recorded (FFS_LDS_AUTO's sizing).
template <int MAXM>
__global__ __launch_bounds__(64) void overflow_kernel(DInst I, const int32_t *__restrict__ prio,
                                                      int64_t *obj, int64_t *work, int32_t *start,
                                                      int32_t *mach, Header *hdr,
                                                      const int32_t *ovf_list, uint8_t *gprof,
                                                      size_t gstride, int32_t *span) {
  extern __shared__ __align__(16) uint8_t smem[];
  Lds l = carve_lds(smem, I.n);
  const int count = __hip_atomic_load(&hdr->ovf_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  GlobalProfile prof{gprof + gstride * blockIdx.x, offchip_cap(I.horizon)};
  for (int e = blockIdx.x; e < count; e += gridDim.x) {
    const int i = uni(ovf_list[e]);
    const int32_t *src = prio + (size_t)i * I.n;
    for (int k = __lane_id(); k < I.n; k += kWave) l.gene[k] = src[k];
    __asm__ volatile("" ::: "memory");
    const size_t plan = (size_t)i * I.n_jobs * I.g;
    int64_t w = 0;
    int64_t *wp = work ? work + i : &w;
    const int st = start ? decode_core<MAXM, true>(I, l, prof, obj + i, wp, start + plan, mach + plan,
                                                   span)
                         : decode_core<MAXM, false>(I, l, prof, obj + i, wp, nullptr, nullptr, span);
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
  // An off-chip profile per individual (redo_stride bytes each) for redoing
  // its own overflowed decode; null when the overflow kernel does the redo.
  uint8_t *redo_prof;
  size_t redo_stride;
  u64 seed, shop;
  // islands: the islands a generation launch covers, from island isl0 on (the
  // whole population but for ga_step's island groups); narrow: the generation
  // and init kernels take the narrow LDS layout (LdsN)
  int32_t event, rows, cols, islands, mig_k, isl0, narrow;
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
// first_pos: LDS [n + 1], miss: LDS [n] (16-bit words when n < 65536).
template <class M>
__device__ void correct_lds(int32_t *gene, int n, int32_t *first_pos, M *miss) {
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
    const u64 m = ballot64(missing);
    if (missing) miss[rank + __popcll(m & below)] = (M)v;
    rank += __popcll(m);
  }
  __asm__ volatile("" ::: "memory");
  rank = 0;
  for (int b = 0; b < n; b += kWave) {
    const int k = b + lane;
    const int v = k < n ? gene[k] : 1;
    const bool dup = k < n && (v < 1 || v > n || first_pos[v] != k);
    const u64 m = ballot64(dup);
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

// Build slot i's child in l.gene (and store it in A.prio_out unless !store) from
// its parent `mine` and, when cross_idx >= 0, the partner parent `other`:
// slot cross_idx's purpose-1 block decides the crossover (p_c) and its cut, the
// child is mine's head and other's tail, corrected (Fig. 11); then slot i's
// purpose-2 block decides the swap mutation (Fig. 12). Both Philox blocks are
// evaluated together on two lanes (the scalar unit, which the CU's waves
// share, is the busier one). Every lane calls this.
template <class L>
__device__ void build_child(const GaDev &A, int n, int i, int gen, const L &l,
                            const int32_t *mine, const int32_t *other, int cross_idx,
                            int variant, bool store) {
  const int lane = __lane_id();
  int32_t *first_pos = scratch32(l);  // free before the decode
  uint16_t *miss = scratch16(l);
  u64 dw[4];
  {
    const bool xl = lane == 0;
    philox((u64)(xl ? cross_idx : i), (u64)gen, (u64)A.event,
           ((xl ? 1ull : 2ull) << 32) | (u64)variant, A.seed, A.shop, dw);
  }
  const uint32_t xw0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[0] >> 32), 0);
  const uint32_t xw1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[1] >> 32), 0);
  const uint32_t mw0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[0] >> 32), 1);
  const uint32_t mw1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[1] >> 32), 1);
  const uint32_t mw2 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[2] >> 32), 1);
  bool cross = false;
  int cut = n;
  if (cross_idx >= 0 && n >= 2) {
    cross = xw0 < A.pc;
    cut = 1 + (int)draw_below((u64)xw1 << 32, (uint32_t)(n - 1));
  }
  if (cross) {
    for (int k = lane; k < n; k += kWave) l.gene[k] = k < cut ? mine[k] : other[k];
    __asm__ volatile("" ::: "memory");
    correct_lds(l.gene, n, first_pos, miss);
  } else {
    for (int k = lane; k < n; k += kWave) l.gene[k] = mine[k];
    __asm__ volatile("" ::: "memory");
  }
  if (n >= 2) {  // swap mutation (Fig. 12)
    if (mw0 < A.pm) {
      const int x = (int)draw_below((u64)mw1 << 32, (uint32_t)n);
      int y = (int)draw_below((u64)mw2 << 32, (uint32_t)(n - 1));
      y += y >= x;
      if (lane == 0) {
        const int gx = l.gene[x];
        l.gene[x] = l.gene[y];
        l.gene[y] = gx;
      }
      __asm__ volatile("" ::: "memory");
    }
  }
  if (!store) return;
  int32_t *dst = A.prio_out + (size_t)i * n;
  for (int k = lane; k < n; k += kWave) dst[k] = l.gene[k];
}

// Build the child of slot i for generation gen in l.gene (and store it in
// A.prio_out): local selection of both parents, neighbour-paired crossover
// with correction, swap mutation. Crossover and mutation draw from Philox
// block `variant` (0 for the plain generation; the screened generation's
// candidates use 0..V-1). Every lane calls this.
template <class L>
__device__ void breed_child(const GaDev &A, int n, int i, int gen, const L &l, int variant = 0,
                            bool store = true) {
  const int K = A.rows * A.cols;
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
  const int32_t *mine = A.prio_in + (size_t)select_winner(A, i) * n;
  const int32_t *other = lead >= 0 ? A.prio_in + (size_t)select_winner(A, partner) * n : mine;
  build_child(A, n, i, gen, l, mine, other, lead, variant, store);
}

// Generation 0 of slot i: Fisher-Yates over 1..n, draw d from word d % 4 of
// block d / 4 of purpose 0; the result goes to l.gene and A.prio_out.
template <class L>
__device__ void init_child(const GaDev &A, int n, int i, const L &l) {
  const int lane = __lane_id();
  uint32_t *hi = (uint32_t *)scratch32(l);  // n - 1 high words (scratch before the decode)
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
}

// Decode l.gene for slot i (its genes are also in A.prio_out) and record the
// outcome: the objective, the work count, or an overflow entry `tag` for the
// off-chip redo, which the wave does itself when it has a profile of its own
// (in the wide layout, laid over the same LDS: both start at rdy).
template <int MAXM, class L>
__device__ void decode_and_record(const DInst &I, const GaDev &A, int i, int cap, const L &l,
                                  int tag, int32_t *span = nullptr) {
  int64_t work = 0;
  int st = decode_core<MAXM, false>(I, l, LdsProfile{l.prof, cap}, A.obj_out + i, &work, nullptr,
                                    nullptr, span);
  // a schedule longer than the on-chip slots: at least cap + 1 of them
  if (st == kDecOverflow && __lane_id() == 0) {
    atomicAdd(&A.hdr->overflows, 1ull);
    if (span) atomicMax(span, cap + 1);
  }
  if (st == kDecOverflow && A.redo_prof) {
    const Lds lw = carve_lds((uint8_t *)l.rdy, I.n);
    const int32_t *src = A.prio_out + (size_t)i * I.n;
    for (int k = __lane_id(); k < I.n; k += kWave) lw.gene[k] = src[k];  // this lane's own stores
    __asm__ volatile("" ::: "memory");
    work = 0;
    const GlobalProfile gp{A.redo_prof + A.redo_stride * i, offchip_cap(I.horizon)};
    st = decode_core<MAXM, false>(I, lw, gp, A.obj_out + i, &work, nullptr, nullptr, span);
    if (st == kDecOverflow) st = kDecInval;  // the horizon bound was wrong: cannot happen
  }
  if (st == kDecOk) {
    if (__lane_id() == 0) atomicAdd(&A.hdr->work, (unsigned long long)work);
    return;
  }
  if (__lane_id() == 0) A.obj_out[i] = -1;
  if (st == kDecOverflow) push_overflow(A.hdr, A.ovf_list, tag);
  else flag_error(A.hdr, st);
}

template <bool MAX>
__device__ void wave_arg(int64_t &v, int &idx) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const int64_t ov = __shfl_xor(v, d, kWave);
    const int oi = __shfl_xor(idx, d, kWave);
    const bool take = MAX ? (ov > v || (ov == v && oi < idx)) : (ov < v || (ov == v && oi < idx));
    if (take) {
      v = ov;
      idx = oi;
    }
  }
}

// Replacement of island I by one wave (same rule as replace_island): the best
// child becomes the best-in-history if it beats it, and the best-in-history
// replaces the worst child. The genes kept are read once and stored to both
// places (a slot that is both best and worst gets its own genes back).
__device__ void replace_island_wave(const GaDev &A, int I, int K, int n) {
  const int lane = __lane_id(), base = I * K;
  const int64_t old = A.elite_obj[I];  // read beside the objectives
  int64_t bv = LLONG_MAX, wv = LLONG_MIN;
  int b = INT_MAX, w = INT_MAX;
  for (int k = lane; k < K; k += kWave) {
    const int64_t o = A.obj_out[base + k];
    if (o < bv) {
      bv = o;
      b = k;
    }
    if (o > wv) {
      wv = o;
      w = k;
    }
  }
  wave_arg<false>(bv, b);
  wave_arg<true>(wv, w);
  const bool better = bv < old;
  int32_t *elite = A.elite + (size_t)I * n, *worst = A.prio_out + (size_t)(base + w) * n;
  const int32_t *keep = better ? A.prio_out + (size_t)(base + b) * n : elite;
  for (int k = lane; k < n; k += kWave) {
    const int32_t v = keep[k];
    if (better) elite[k] = v;
    worst[k] = v;
  }
  if (lane == 0) {
    if (better) A.elite_obj[I] = bv;
    A.obj_out[base + w] = better ? bv : old;
  }
}


// ---------------------------------------------------------------------------
// The comparison GAs of Section 5.2 on job-priority vectors, one population of
// rows x cols individuals (islands = 1): the classical GA (roulette wheel on
// eq. (13)'s fitness, random pairing) and the cellular GA (parents from the
// neighbourhood, replace if better).
// ---------------------------------------------------------------------------
// E_max of eq. (13): 10^a, the least a >= 1 above every objective of generation 0.
__global__ __launch_bounds__(256) void emax_kernel(const int64_t *obj, int pop, Header *h) {
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  int64_t m = LLONG_MIN;
  for (int i = t; i < pop; i += 256) m = max(m, obj[i]);
  sh[t] = m;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sh[t] = max(sh[t], sh[t + w]);
    __syncthreads();
  }
  if (t == 0) {
    int64_t e = 10;
    while (!(sh[0] < e) && e <= LLONG_MAX / 10) e *= 10;
    h->e_max = e;
  }
}

// Running sums of eq. (13)'s fitness F_i = max(E_max - obj_i, 0) in index
// order (integers: any order of additions gives the same sums). Thread t of
// one block of 1024 sums a run of consecutive entries; the runs' totals are
// scanned and each run then writes its running sums.
__global__ __launch_bounds__(1024) void fitness_scan_kernel(const int64_t *obj, int pop,
                                                            const Header *h, u64 *prefix) {
  __shared__ u64 part[1024];
  const int t = threadIdx.x;
  const int64_t e = h->e_max;
  const int c = (pop + 1023) / 1024;
  const int a = min(t * c, pop), b = min(a + c, pop);
  u64 sum = 0;
  for (int i = a; i < b; ++i) {
    const int64_t f = e - obj[i];
    sum += f > 0 ? (u64)f : 0ull;
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const u64 v = t >= d ? part[t - d] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  u64 run = t > 0 ? part[t - 1] : 0ull;
  for (int i = a; i < b; ++i) {
    const int64_t f = e - obj[i];
    run += f > 0 ? (u64)f : 0ull;
    prefix[i] = run;
  }
}

// Roulette spin of slot s (word 0 of its purpose-6 block): the first
// individual whose running fitness sum exceeds floor(hi32 * total / 2^32), a
// uniform one when every fitness is 0. The wave narrows the range 64-fold per
// step, each lane testing the last running sum of one of 64 sub-ranges (the
// first sub-range whose last sum exceeds the target holds the answer).
__device__ int roulette_spin(const GaDev &A, const u64 *prefix, int pop, int s, int gen) {
  u64 w[4];
  philox((u64)s, (u64)gen, (u64)A.event, 6ull << 32, A.seed, A.shop, w);
  const u64 total = prefix[pop - 1];
  if (total == 0) return (int)draw_below(w[0], (uint32_t)pop);
  const u64 target = __umul64hi((w[0] >> 32) << 32, total);
  const int lane = __lane_id();
  int lo = 0, hi = pop;  // the answer lies in [lo, hi) and prefix[hi - 1] > target
  while (hi - lo > kWave) {
    const int step = (hi - lo + kWave - 1) / kWave;
    const int e = min(lo + (lane + 1) * step, hi) - 1;
    const u64 m = ballot64(prefix[e] > target);
    const int f = __ffsll((long long)m) - 1;
    const int nlo = lo + f * step;
    hi = min(nlo + step, hi);
    lo = nlo;
  }
  const u64 m = ballot64(lo + lane < hi && prefix[min(lo + lane, hi - 1)] > target);
  return lo + __ffsll((long long)m) - 1;
}

// Classical GA, one wave per slot: the slot's and its pair partner's parents by
// roulette, the pair (2k, 2k+1) crossing at slot 2k's cut, swap mutation, decode.
template <int MAXM>
__global__ __launch_bounds__(64) void classical_generation_kernel(DInst I, GaDev A, int gen,
                                                                  int cap, const u64 *prefix) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x, pop = A.rows * A.cols, partner = i ^ 1;
  const Lds l = carve_lds(smem, I.n);
  const int32_t *mine = A.prio_in + (size_t)roulette_spin(A, prefix, pop, i, gen) * I.n;
  if (partner < pop) {
    const int32_t *other = A.prio_in + (size_t)roulette_spin(A, prefix, pop, partner, gen) * I.n;
    build_child(A, I.n, i, gen, l, mine, other, i & ~1, 0, true);
  } else {
    build_child(A, I.n, i, gen, l, mine, mine, -1, 0, true);
  }
  decode_and_record<MAXM>(I, A, i, cap, l, i);
}

// Cellular GA, one wave per cell: the best two of the cell and its four torus
// neighbours (by objective, then in the order self, up, down, left, right),
// crossing at the cell's own cut, swap mutation, decode.
template <int MAXM>
__global__ __launch_bounds__(64) void cellular_generation_kernel(DInst I, GaDev A, int gen,
                                                                 int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x, R = A.rows, C = A.cols, r = i / C, c = i % C;
  const Lds l = carve_lds(smem, I.n);
  const int cand[5] = {i, ((r + R - 1) % R) * C + c, ((r + 1) % R) * C + c,
                       r * C + (c + C - 1) % C, r * C + (c + 1) % C};
  int64_t o[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) o[k] = ld_const(A.obj_in, (size_t)cand[k]);
  int b1 = 0, b2 = -1;
#pragma unroll
  for (int k = 1; k < 5; ++k)
    if (o[k] < o[b1]) b1 = k;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (k != b1 && (b2 < 0 || o[k] < o[b2])) b2 = k;
  build_child(A, I.n, i, gen, l, A.prio_in + (size_t)cand[b1] * I.n,
              A.prio_in + (size_t)cand[b2] * I.n, i, 0, true);
  decode_and_record<MAXM>(I, A, i, cap, l, i);
}

// Cellular replacement: a cell keeps its previous individual unless the child
// is strictly better (one wave per cell, after any off-chip redo).
__global__ __launch_bounds__(64) void cellular_accept_kernel(const int32_t *prio_in,
                                                             const int64_t *obj_in,
                                                             int32_t *prio_out, int64_t *obj_out,
                                                             int n) {
  const int i = blockIdx.x;
  if (obj_out[i] < obj_in[i]) return;
  for (int k = __lane_id(); k < n; k += kWave) prio_out[(size_t)i * n + k] = prio_in[(size_t)i * n + k];
  if (__lane_id() == 0) obj_out[i] = obj_in[i];
}

// Best in history of a whole population (lowest objective, lowest slot on ties).
__global__ __launch_bounds__(64) void elite_update_kernel(const int32_t *prio, const int64_t *obj,
                                                          int32_t *elite, int64_t *elite_obj,
                                                          int pop, int n) {
  int64_t bv = LLONG_MAX;
  int b = INT_MAX;
  for (int k = __lane_id(); k < pop; k += kWave) {
    const int64_t o = obj[k];
    if (o < bv) {
      bv = o;
      b = k;
    }
  }
  wave_arg<false>(bv, b);
  if (bv < elite_obj[0]) {
    for (int k = __lane_id(); k < n; k += kWave) elite[k] = prio[(size_t)b * n + k];
    if (__lane_id() == 0) elite_obj[0] = bv;
  }
}

template <int MAXM>
__global__ __launch_bounds__(64) void ga_generation_kernel(DInst I, GaDev A, int gen, int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int K = A.rows * A.cols;
  const int i = A.isl0 * K + slot_of_block(blockIdx.x, K, A.islands);
  if (A.narrow) {  // the narrow layout (lds_bytes_n): default rules only
    const LdsN l = carve_lds_n(smem, I.n);
    breed_child(A, I.n, i, gen, l);
    decode_and_record<MAXM>(I, A, i, cap, l, i);
  } else {
    const Lds l = carve_lds(smem, I.n);
    breed_child(A, I.n, i, gen, l);
    decode_and_record<MAXM>(I, A, i, cap, l, i);
  }
}

// Generation 0. span: null, or where the longest schedule is recorded
// (ga_init sizes the on-chip profile of later generations from it).
template <int MAXM>
__global__ __launch_bounds__(64) void ga_init_kernel(DInst I, GaDev A, int cap, int32_t *span) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x;
  if (A.narrow) {  // the narrow layout (lds_bytes_n): default rules only
    const LdsN l = carve_lds_n(smem, I.n);
    init_child(A, I.n, i, l);
    decode_and_record<MAXM>(I, A, i, cap, l, i, span);
  } else {
    const Lds l = carve_lds(smem, I.n);
    init_child(A, I.n, i, l);
    decode_and_record<MAXM>(I, A, i, cap, l, i, span);
  }
}

// LDS of the generation and init kernels in the layout they take.
size_t lds_bytes_gen(const ffs_instance *in, int cap, bool narrow) {
  return narrow ? lds_bytes_n(in->n_active, cap) : lds_bytes(in->n_active, cap);
}

// ---------------------------------------------------------------------------
// The paper's own chromosome: target machines X and operation priorities Y
// (Section 4.3, eqs. (10)-(12)). Only unfrozen ops carry genes, R of them,
// row-major over the active jobs (gene k <-> op xyop[k] = x | s << 20 of
// active job x, with the stage's machine count o_s as (o_s - 1) << 27; job x's
// genes are [xyg0[x], xyg0[x+1])). A chromosome is
// 2R ints: the R machines, then the R priorities (a permutation of 1..R,
// larger = higher).
// ---------------------------------------------------------------------------
struct XyTab {
  const int32_t *op;   // [R]: x | s << 20 | (o_s - 1) << 27
  const int32_t *g0;   // [n + 1]
  int32_t R;
};

// LDS of one wave decoding an X/Y chromosome:
//   gx   [R]      machine genes
//   zrec [R+1]    ops in Z order: (x | (s * om + m) << 12, P|Q) for active job x,
//                 then a zero record the op loop reads one past the last
//   rdy  [n]      completion of each active job's last placed stage
//   fm   [g*om]   machine free times (rdy and fm live in registers instead
//                 when there are at most 128 jobs and 64 machine slots)
//   then one region used twice: until Z is built, the priority genes gy [R]
//   (once the heads are built, each gene's place in Z)
//   and head [R+1] (per priority value y: k | len << 24 when gene k starts a
//   chain of len genes of one job whose running minimum of y is y, else 0);
//   from then on the power profile prof [cap+64]. A decode redone off chip
//   therefore reloads its genes.
// head and zrec double as the breeding scratch (correction, Fisher-Yates).
struct LdsXy {
  int32_t *gx, *gy;
  int32_t *head;
  int2 *zrec;
  int32_t *rdy, *fm;
  uint8_t *prof;
};

__host__ __device__ inline size_t lds_bytes_xy(int n, int R, int g, int om, int cap) {
  const size_t genes = 2 * align_up((size_t)4 * R + 4, 16);
  const size_t prof = cap > 0 ? align_up(cap, 16) + kWave : 0;
  return align_up((size_t)4 * R + 4, 16) + align_up((size_t)8 * R + 8, 16) +
         align_up((size_t)4 * n + 4, 16) + align_up((size_t)4 * g * om, 16) +
         (genes > prof ? genes : prof);
}

__device__ __forceinline__ LdsXy carve_lds_xy(uint8_t *smem, int n, int R, int g, int om) {
  LdsXy l;
  size_t off = 0;
  l.gx = (int32_t *)(smem + off);
  off += align_up((size_t)4 * R + 4, 16);
  l.zrec = (int2 *)(smem + off);
  off += align_up((size_t)8 * R + 8, 16);
  l.rdy = (int32_t *)(smem + off);
  off += align_up((size_t)4 * n + 4, 16);
  l.fm = (int32_t *)(smem + off);
  off += align_up((size_t)4 * g * om, 16);
  l.gy = (int32_t *)(smem + off);
  l.head = (int32_t *)(smem + off + align_up((size_t)4 * R + 4, 16));
  l.prof = smem + off;
  return l;
}

// Inclusive prefix sum over the 64 lanes (lane order).
__device__ __forceinline__ int wave_scan_incl(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Decode the X/Y chromosome in l.gx / l.gy (Algorithms 1 and 2). Z: the greedy
// order of Algorithm 1 (the op of largest y among each job's next unordered
// op) equals the ops sorted by the running minimum of y along each job's
// stages, descending, ties (same job) by stage: each job splits into chains
// that start where the running minimum drops, and the chains go out by their
// head's y, highest first. Each op then goes on its machine x at the
// earliest power-feasible start after its job's previous stage and the
// machine's last op, as in decode_core. Every lane calls this; the result is
// uniform; on kDecOk lane 0 has written *obj_out.
//
// NB = 1 or 2: the jobs' ready times and the machines' free times live in
// registers (lane x of rv0 / rv1 holds job x / 64 + x, lane f of fmv machine
// f), read with readlane and written with writelane, so an op waits on no LDS
// read but its profile chunk; needs at most 64 * NB active jobs and 64 machine
// slots (g * o_max). NB = 0: they live in LDS and are read one op ahead.
template <bool PLAN, int NB, class Prof>
__device__ int decode_xy_core_t(const DInst &I, const XyTab &T, const LdsXy &l, Prof &&prof,
                                int64_t *obj_out, int64_t *work_out, int32_t *start_out,
                                int32_t *mach_out) {
  const int lane = __lane_id(), n = I.n, R = T.R;
  for (int y = lane; y <= R; y += kWave) l.head[y] = 0;
  __asm__ volatile("" ::: "memory");
  // x genes name a machine of their stage; y genes are a permutation of 1..R
  // (each value counted once)
  int bad = 0;
  for (int k = lane; k < R; k += kWave) {
    const int x = l.gx[k], os = (ld_const(T.op, k) >> 27) + 1;
    if (x < 0 || x >= os) bad = 1;
    const int y = l.gy[k];
    if (y < 1 || y > R) bad = 1;
    else atomicAdd(&l.head[y], 1);
  }
  __asm__ volatile("" ::: "memory");
  for (int y = 1 + lane; y <= R; y += kWave) bad |= l.head[y] != 1;
  if (ballot64(bad)) return kDecInval;
  for (int y = lane; y <= R; y += kWave) l.head[y] = 0;
  __asm__ volatile("" ::: "memory");
  // chain heads, one job per lane
  for (int x = lane; x < n; x += kWave) {
    const int k0 = ld_const(T.g0, x), k1 = ld_const(T.g0, x + 1);
    int hk = -1, m = INT_MAX;
    for (int k = k0; k < k1; ++k) {
      const int y = l.gy[k];
      if (y < m) {
        if (hk >= 0) l.head[m] = hk | (k - hk) << 24;
        hk = k;
        m = y;
      }
    }
    if (hk >= 0) l.head[m] = hk | (k1 - hk) << 24;
  }
  __asm__ volatile("" ::: "memory");
  // Z: chains by decreasing head value. First each gene's place in Z (into the
  // priority genes' words, dead once the heads are built: LDS only), then each
  // op's record, one gene per lane, so the table reads of different genes are
  // in flight together instead of one chain element after another.
  int32_t *zpos = l.gy;
  int base = 0;
  for (int y0 = R; y0 >= 1; y0 -= kWave) {
    const int y = y0 - lane;
    const int h = y >= 1 ? l.head[y] : 0;
    const int len = (int)((uint32_t)h >> 24), k = h & 0xFFFFFF;
    const int incl = wave_scan_incl(len);
    const int pos = base + incl - len;
    for (int i = 0; i < len; ++i) zpos[k + i] = pos + i;
    base += __builtin_amdgcn_readlane(incl, kWave - 1);
  }
  __asm__ volatile("" ::: "memory");
  for (int kk = lane; kk < R; kk += kWave) {
    const int op = ld_const(T.op, kk), x = op & 0xFFFFF, s = (op >> 20) & 0x7F;
    const int m = l.gx[kk];
    const uint32_t pq = ld_const(I.pq, ((size_t)x * I.g + s) * I.omp + m);
    l.zrec[zpos[kk]] = make_int2(x | (s * I.om + m) << 12, (int)pq);
  }
  if (lane == 0) l.zrec[R] = make_int2(0, 0);  // spare record: the loop reads one past the last
  int rv0 = 0, rv1 = 0, fmv = 0;
  if constexpr (NB > 0) {
    if (lane < n) rv0 = ld_const(I.ready, ld_const(I.active, lane));
    if (NB > 1 && kWave + lane < n) rv1 = ld_const(I.ready, ld_const(I.active, kWave + lane));
    if (lane < I.g * I.om) fmv = ld_const(I.mfree, lane);
  } else {
    for (int x = lane; x < n; x += kWave) l.rdy[x] = ld_const(I.ready, ld_const(I.active, x));
    for (int x = lane; x < I.g * I.om; x += kWave) l.fm[x] = ld_const(I.mfree, x);
  }
  prof.clear();
  prof.order();
  for (int r = 0; r < I.nr; ++r) {
    const int len = ld_const(I.running, 2 * r) - I.rs;
    if (len > prof.cap) return kDecOverflow;
    prof.add_running(len, ld_const(I.running, 2 * r + 1));
  }
  for (int r = 0; r < I.nf; ++r) {
    const int b = ld_const(I.fixed, 3 * r + 1) - I.rs;
    if (b > prof.cap) return kDecOverflow;
    prof.add_span(ld_const(I.fixed, 3 * r) - I.rs, b, ld_const(I.fixed, 3 * r + 2));
  }
  prof.order();
  __asm__ volatile("" ::: "memory");

  // Ops in Z order, the next op's record read one op ahead.
  const int rs = I.rs, cap = prof.cap;
  int64_t work = 0;
  int max_end = rs;
  int2 rec = R > 0 ? l.zrec[0] : make_int2(0, 0);
  if constexpr (NB > 0) {
    uint64_t wsum;  // per lane: summed on the vector unit
    const int2 *zp;  // per lane too: records read with immediate offsets
    {
      int vz;
      __asm__("v_mov_b32 %0, 0" : "=v"(vz));
      wsum = (uint64_t)(uint32_t)vz;
      zp = l.zrec + vz;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // as in decode_core_rules: no wait at the loop's head
    // each op's profile update issued by the next op, as in decode_core_rules
    int ct = 0, cp = 0, cq = 0;
    for (int z = 0; z < R; ++z) {
      const int xf = uni(rec.x), x = xf & 0xFFF, f = xf >> 12, pqw = uni(rec.y);
      rec = *++zp;
      const int xl = x & (kWave - 1);
      // both registers read and written, the right one chosen: no branch
      const int r0 = __builtin_amdgcn_readlane(rv0, xl);
      const int r1 = NB > 1 ? __builtin_amdgcn_readlane(rv1, xl) : 0;
      const bool hi = NB > 1 && x >= kWave;
      const int est = max(rs, hi ? r1 : r0), fr = __builtin_amdgcn_readlane(fmv, f);
      const int p = pqw & 0xFFFF, q = (int)((uint32_t)pqw >> 16);
      const int t0 = max(est, fr) - rs;
      prof.commit(ct, cp, cq);
      const int t = prof.place(t0, p, (uint32_t)(I.q_max - q));
      ct = t;
      cp = p;
      cq = q;
      const int end = t + p + rs;
      rv0 = ffs_writelane(hi ? r0 : end, xl, rv0);
      if (NB > 1) rv1 = ffs_writelane(hi ? end : r1, xl, rv1);
      fmv = ffs_writelane(end, f, fmv);
      wsum += (uint32_t)((t - t0) + 2 * p);  // non-negative
      max_end = max(max_end, end);
      if (PLAN && lane == 0) {
        const int j = ld_const(I.active, x), s = f / I.om;
        start_out[(size_t)j * I.g + s] = t + rs;
        mach_out[(size_t)j * I.g + s] = f - s * I.om;
      }
    }
    prof.commit(ct, cp, cq);
    work = (int64_t)(((uint64_t)(uint32_t)uni((int)(uint32_t)(wsum >> 32)) << 32) |
                     (uint32_t)uni((int)(uint32_t)wsum));
    if (lane < n) l.rdy[lane] = rv0;
    if (NB > 1 && kWave + lane < n) l.rdy[kWave + lane] = rv1;
  } else {
    // The next op's job-ready and machine-free times are read one op ahead too;
    // an op that frees the next op's job or machine hands its end over directly.
    int rdy_n = l.rdy[uni(rec.x) & 0xFFF], fm_n = l.fm[uni(rec.x) >> 12];
    for (int z = 0; z < R; ++z) {
      const int xf = uni(rec.x), x = xf & 0xFFF, f = xf >> 12, pqw = uni(rec.y);
      const int est = max(rs, uni(rdy_n)), fr = uni(fm_n);
      rec = l.zrec[z + 1];
      const int xfn = uni(rec.x), xn = xfn & 0xFFF, fn = xfn >> 12;
      rdy_n = l.rdy[xn];
      fm_n = l.fm[fn];
      const int p = pqw & 0xFFFF, q = (int)((uint32_t)pqw >> 16);
      const uint32_t thr = (uint32_t)(I.q_max - q);
      const int t0 = max(est, fr) - rs;
      const int t = prof.place(t0, p, thr);
      prof.commit(t, p, q);
      const int end = t + p + rs;
      l.rdy[x] = end;
      l.fm[f] = end;
      if (xn == x) rdy_n = end;
      if (fn == f) fm_n = end;
      work += (int64_t)(t - t0) + 2 * p;
      max_end = max(max_end, end);
      if (PLAN && lane == 0) {
        const int j = ld_const(I.active, x), s = f / I.om;
        start_out[(size_t)j * I.g + s] = t + rs;
        mach_out[(size_t)j * I.g + s] = f - s * I.om;
      }
    }
  }
  if (max_end - rs > cap) return kDecOverflow;
  __asm__ volatile("" ::: "memory");
  int64_t tard = 0;
  int cmax = 0;
  for (int x = lane; x < n; x += kWave) {
    const int c = l.rdy[x];
    const int late = c - ld_const(I.due_k, x);
    tard += late > 0 ? late : 0;
    cmax = max(cmax, c);
  }
  tard = wave_sum64(tard);
  cmax = max(wave_max32(cmax), I.frozen_cmax);
  if (lane == 0) {
    *obj_out = (int64_t)I.wt * (I.frozen_t + tard) + cmax;
    if (work_out) *work_out = work;
  }
  return kDecOk;
}

template <bool PLAN, class Prof>
__device__ __forceinline__ int decode_xy_core(const DInst &I, const XyTab &T, const LdsXy &l,
                                              Prof &&prof, int64_t *obj_out, int64_t *work_out,
                                              int32_t *start_out, int32_t *mach_out) {
  if (I.g * I.om <= kWave && I.n <= kWave)
    return decode_xy_core_t<PLAN, 1>(I, T, l, prof, obj_out, work_out, start_out, mach_out);
  if (I.g * I.om <= kWave && I.n <= 2 * kWave)
    return decode_xy_core_t<PLAN, 2>(I, T, l, prof, obj_out, work_out, start_out, mach_out);
  return decode_xy_core_t<PLAN, 0>(I, T, l, prof, obj_out, work_out, start_out, mach_out);
}

// Gene/op table of an instance (one block of 1024 threads): the active jobs'
// gene offsets by a block prefix sum, then each gene's (x, stage, machines of
// the stage), so a gene's machine range needs no second read.
__global__ __launch_bounds__(1024) void xy_table_kernel(const int32_t *first, const int32_t *active,
                                                        const int32_t *nm, int n, int g,
                                                        int32_t *op, int32_t *g0) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x, per = (n + 1023) / 1024, x0 = t * per, x1 = min(n, x0 + per);
  int sum = 0;
  for (int x = x0; x < x1; ++x) sum += g - first[active[x]];
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int k = part[t] - sum;
  for (int x = x0; x < x1; ++x) {
    g0[x] = k;
    for (int s = first[active[x]]; s < g; ++s)
      op[k++] = x | s << 20 | (min(max(nm[s], 1), 16) - 1) << 27;  // 1 <= o_s <= 16
  }
  if (t == 1023) g0[n] = part[1023];
}

template <int MAXM>
__global__ __launch_bounds__(64) void decode_xy_kernel(DInst I, XyTab T, const int32_t *__restrict__ genes,
                                                       int64_t *obj, int64_t *work, int32_t *start,
                                                       int32_t *mach, Header *hdr, int32_t *ovf_list,
                                                       int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x;
  const LdsXy l = carve_lds_xy(smem, I.n, T.R, I.g, I.om);
  const int32_t *src = genes + (size_t)i * 2 * T.R;
  for (int k = __lane_id(); k < T.R; k += kWave) {
    l.gx[k] = src[k];
    l.gy[k] = src[T.R + k];
  }
  __asm__ volatile("" ::: "memory");
  const size_t plan = (size_t)i * I.n_jobs * I.g;
  const LdsProfile prof{l.prof, cap};
  int64_t *w = work ? work + i : nullptr;
  const int st = start ? decode_xy_core<true>(I, T, l, prof, obj + i, w, start + plan, mach + plan)
                       : decode_xy_core<false>(I, T, l, prof, obj + i, w, nullptr, nullptr);
  if (st == kDecOk) return;
  if (__lane_id() == 0) obj[i] = -1;
  if (st == kDecOverflow) push_overflow(hdr, ovf_list, i);
  else flag_error(hdr, st);
}

// Redo of overflowed X/Y decodes with a global-memory profile (as overflow_kernel).
template <int MAXM>
__global__ __launch_bounds__(64) void overflow_xy_kernel(DInst I, XyTab T, const int32_t *__restrict__ genes,
                                                         int64_t *obj, int64_t *work, int32_t *start,
                                                         int32_t *mach, Header *hdr,
                                                         const int32_t *ovf_list, uint8_t *gprof,
                                                         size_t gstride) {
  extern __shared__ __align__(16) uint8_t smem[];
  const LdsXy l = carve_lds_xy(smem, I.n, T.R, I.g, I.om);
  const int count = __hip_atomic_load(&hdr->ovf_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  GlobalProfile prof{gprof + gstride * blockIdx.x, offchip_cap(I.horizon)};
  for (int e = blockIdx.x; e < count; e += gridDim.x) {
    const int i = uni(ovf_list[e]);
    const int32_t *src = genes + (size_t)i * 2 * T.R;
    for (int k = __lane_id(); k < T.R; k += kWave) {
      l.gx[k] = src[k];
      l.gy[k] = src[T.R + k];
    }
    __asm__ volatile("" ::: "memory");
    const size_t plan = (size_t)i * I.n_jobs * I.g;
    int64_t w = 0;
    int64_t *wp = work ? work + i : &w;
    const int st = start ? decode_xy_core<true>(I, T, l, prof, obj + i, wp, start + plan, mach + plan)
                         : decode_xy_core<false>(I, T, l, prof, obj + i, wp, nullptr, nullptr);
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

// Generation 0 of slot i for an X/Y chromosome: each x a uniform machine of
// its stage (word k % 4 of block k / 4 of purpose 4), y by Fisher-Yates over
// 1..R as init_child does (purpose 0); stored to A.prio_out (2R ints).
__device__ void init_child_xy(const GaDev &A, const DInst &I, const XyTab &T, int i,
                              const LdsXy &l) {
  const int lane = __lane_id(), R = T.R;
  for (int b = lane; b < (R + 3) / 4; b += kWave) {
    u64 w[4];
    philox((u64)i, 0ull, (u64)A.event, (4ull << 32) | (u64)b, A.seed, A.shop, w);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * b + u;
      if (k < R) l.gx[k] = (int)draw_below(w[u], (uint32_t)(ld_const(T.op, k) >> 27) + 1u);
    }
  }
  uint32_t *hi = (uint32_t *)l.zrec;  // R - 1 high words
  for (int k = lane; k < R; k += kWave) l.gy[k] = k + 1;
  for (int b = lane; b < (R - 1 + 3) / 4; b += kWave) {
    u64 w[4];
    philox((u64)i, 0ull, (u64)A.event, (u64)b, A.seed, A.shop, w);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (4 * b + u < R - 1) hi[4 * b + u] = (uint32_t)(w[u] >> 32);
  }
  __asm__ volatile("" ::: "memory");
  if (lane == 0) {
    for (int pos = R - 1; pos >= 1; --pos) {
      const int r = (int)(((u64)hi[R - 1 - pos] * (u64)(pos + 1)) >> 32);
      const int t = l.gy[pos];
      l.gy[pos] = l.gy[r];
      l.gy[r] = t;
    }
  }
  __asm__ volatile("" ::: "memory");
  int32_t *dst = A.prio_out + (size_t)i * 2 * R;
  for (int k = lane; k < R; k += kWave) {
    dst[k] = l.gx[k];
    dst[R + k] = l.gy[k];
  }
}

// Child of slot i for generation gen, X/Y chromosome (Section 4.4): local
// selection as breed_child; neighbour-paired single-point crossover cutting
// both matrices at one point (Fig. 11), Y corrected; mutation (Fig. 12) by a
// swap of two y and, with it, every x moved to another machine of its stage,
// (x + 1 + draw(o_s - 1)) mod o_s from word k % 4 of block
// variant * ceil(R / 4) + k / 4 of purpose 5. Stored to A.prio_out.
__device__ void breed_child_xy(const GaDev &A, const DInst &I, const XyTab &T, int i, int gen,
                               const LdsXy &l, int variant = 0) {
  const int lane = __lane_id(), R = T.R, L = 2 * R;
  const int K = A.rows * A.cols;
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
  // crossover block on lane 0, mutation block on the others (as in breed_child)
  u64 dw[4];
  {
    const bool xl = lane == 0;
    philox((u64)(xl ? lead : i), (u64)gen, (u64)A.event,
           ((xl ? 1ull : 2ull) << 32) | (u64)variant, A.seed, A.shop, dw);
  }
  const uint32_t xw0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[0] >> 32), 0);
  const uint32_t xw1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[1] >> 32), 0);
  const uint32_t mw0 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[0] >> 32), 1);
  const uint32_t mw1 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[1] >> 32), 1);
  const uint32_t mw2 = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(dw[2] >> 32), 1);
  const int32_t *mine = A.prio_in + (size_t)select_winner(A, i) * L;
  bool cross = false;
  int cut = R;
  if (lead >= 0 && R >= 2) {
    cross = xw0 < A.pc;
    cut = 1 + (int)draw_below((u64)xw1 << 32, (uint32_t)(R - 1));
  }
  const int32_t *other = cross ? A.prio_in + (size_t)select_winner(A, partner) * L : mine;
  for (int k = lane; k < R; k += kWave) {
    const int32_t *src = k < cut ? mine : other;
    l.gx[k] = src[k];
    l.gy[k] = src[R + k];
  }
  __asm__ volatile("" ::: "memory");
  if (cross) correct_lds(l.gy, R, (int32_t *)l.head, (int32_t *)l.zrec);
  if (mw0 < A.pm) {
    if (R >= 2) {
      const int x = (int)draw_below((u64)mw1 << 32, (uint32_t)R);
      int y = (int)draw_below((u64)mw2 << 32, (uint32_t)(R - 1));
      y += y >= x;
      if (lane == 0) {
        const int gx = l.gy[x];
        l.gy[x] = l.gy[y];
        l.gy[y] = gx;
      }
    }
    const u64 b0 = (u64)variant * (u64)((R + 3) / 4);
    for (int b = lane; b < (R + 3) / 4; b += kWave) {
      u64 v[4];
      philox((u64)i, (u64)gen, (u64)A.event, (5ull << 32) | (b0 + (u64)b), A.seed, A.shop, v);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= R) break;
        const int o = (ld_const(T.op, k) >> 27) + 1;
        if (o > 1) l.gx[k] = (l.gx[k] + 1 + (int)draw_below(v[u], (uint32_t)(o - 1))) % o;
      }
    }
    __asm__ volatile("" ::: "memory");
  }
  int32_t *dst = A.prio_out + (size_t)i * L;
  for (int k = lane; k < R; k += kWave) {
    dst[k] = l.gx[k];
    dst[R + k] = l.gy[k];
  }
}

// decode_and_record for an X/Y chromosome in l (also in A.prio_out, from where
// an off-chip redo reloads it: the on-chip profile overwrote the priorities).
__device__ void decode_and_record_xy(const DInst &I, const XyTab &T, const GaDev &A, int i,
                                     int cap, const LdsXy &l) {
  int64_t work = 0;
  int st = decode_xy_core<false>(I, T, l, LdsProfile{l.prof, cap}, A.obj_out + i, &work, nullptr,
                                 nullptr);
  if (st == kDecOverflow && A.redo_prof) {
    const int32_t *src = A.prio_out + (size_t)i * 2 * T.R;
    for (int k = __lane_id(); k < T.R; k += kWave) {  // this lane's own stores
      l.gx[k] = src[k];
      l.gy[k] = src[T.R + k];
    }
    __asm__ volatile("" ::: "memory");
    work = 0;
    const GlobalProfile gp{A.redo_prof + A.redo_stride * i, offchip_cap(I.horizon)};
    st = decode_xy_core<false>(I, T, l, gp, A.obj_out + i, &work, nullptr, nullptr);
    if (st == kDecOverflow) st = kDecInval;  // the horizon bound was wrong: cannot happen
  }
  if (st == kDecOk) {
    if (__lane_id() == 0) atomicAdd(&A.hdr->work, (unsigned long long)work);
    return;
  }
  if (__lane_id() == 0) A.obj_out[i] = -1;
  if (st == kDecOverflow) push_overflow(A.hdr, A.ovf_list, i);
  else flag_error(A.hdr, st);
}

__global__ __launch_bounds__(64) void ga_init_xy_kernel(DInst I, XyTab T, GaDev A, int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int i = blockIdx.x;
  const LdsXy l = carve_lds_xy(smem, I.n, T.R, I.g, I.om);
  init_child_xy(A, I, T, i, l);
  decode_and_record_xy(I, T, A, i, cap, l);
}

__global__ __launch_bounds__(64) void ga_generation_xy_kernel(DInst I, XyTab T, GaDev A, int gen,
                                                              int cap) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int K = A.rows * A.cols;
  const int i = A.isl0 * K + slot_of_block(blockIdx.x, K, A.islands);
  const LdsXy l = carve_lds_xy(smem, I.n, T.R, I.g, I.om);
  breed_child_xy(A, I, T, i, gen, l);
  decode_and_record_xy(I, T, A, i, cap, l);
}

// Surrogate score of one chromosome (genes 1..n in `gene`, any address
// space): b3 + (sum over k of table[k][gene[k]-1]) / n, summed as 64 lane
// partials over k = lane, lane + 64, ... and then an xor butterfly, lane 0's
// result broadcast. sg_score and the screened generation share this order.
// A gene outside 1..n makes the score NaN (and reads nothing out of range).
__device__ __forceinline__ float score_genes(const int32_t *gene, int n, const float *table,
                                             float b3) {
  const int lane = __lane_id();
  float s = 0.f;
  bool bad = false;
  for (int k = lane; k < n; k += kWave) {
    const int v = gene[k];
    const bool ok = v >= 1 && v <= n;
    bad |= !ok;
    s += table[(size_t)k * n + (ok ? v - 1 : 0)];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  s = __shfl(s, 0);
  if (ballot64(bad)) return __builtin_nanf("");
  return __fadd_rn(b3, __fdiv_rn(s, (float)n));
}

__global__ __launch_bounds__(64) void sg_score_kernel(const float *table, const float *theta,
                                                      int n, const int32_t *prio, float *y) {
  const float s = score_genes(prio + (size_t)blockIdx.x * n, n, table, theta[FFS_SG_PARAMS - 1]);
  if (__lane_id() == 0) y[blockIdx.x] = s;
}

// Screened generation: every cell breeds V candidate children, keeps the one
// with the lowest surrogate score (lowest v on ties), stores and decodes it.
template <int MAXM>
__global__ __launch_bounds__(64) void ga_screened_kernel(DInst I, GaDev A, int gen, int cap,
                                                         const float *table, const float *theta,
                                                         int V, float *scores, int32_t *choice,
                                                         int pop) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int K = A.rows * A.cols;
  const int i = A.isl0 * K + slot_of_block(blockIdx.x, K, A.islands);
  const Lds l = carve_lds(smem, I.n);
  const float b3 = theta[FFS_SG_PARAMS - 1];
  int best = 0;
  float best_s = 0.f;
  for (int v = 0; v < V; ++v) {
    breed_child(A, I.n, i, gen, l, v, false);
    const float sv = score_genes(l.gene, I.n, table, b3);
    if (scores && __lane_id() == 0) scores[(size_t)v * pop + i] = sv;
    if (v == 0 || sv < best_s) {
      best_s = sv;
      best = v;
    }
    __asm__ volatile("" ::: "memory");
  }
  if (choice && __lane_id() == 0) choice[i] = best;
  breed_child(A, I.n, i, gen, l, best, true);
  decode_and_record<MAXM>(I, A, i, cap, l, i);
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
__device__ void replace_island(int32_t *prio, int64_t *obj, int32_t *elite, int64_t *elite_obj,
                               int I, int K, int n, int64_t *sv, int *si) {
  const int base = I * K;
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

// Elitist replacement of every island, one wave per island (replace_island_wave).
__global__ __launch_bounds__(64) void replace_wave_kernel(int32_t *prio, int64_t *obj,
                                                          int32_t *elite, int64_t *elite_obj, int K,
                                                          int n) {
  GaDev A{};
  A.prio_out = prio;
  A.obj_out = obj;
  A.elite = elite;
  A.elite_obj = elite_obj;
  replace_island_wave(A, blockIdx.x, K, n);
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
__device__ void migrate_collect_island(const int32_t *prio, const int64_t *obj,
                                       int32_t *stage_prio, int64_t *stage_obj, int I, int K,
                                       int n, int mig_k, uint8_t *taken, int64_t *sv, int *si) {
  const int base = I * K;
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

__device__ void migrate_apply_island(int32_t *prio, int64_t *obj, int32_t *elite,
                                     int64_t *elite_obj, const int32_t *stage_prio,
                                     const int64_t *stage_obj, int I, int K, int n, int mig_k,
                                     int islands, uint8_t *taken, int64_t *sv, int *si) {
  const int base = I * K, src = (I + islands - 1) % islands;
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

__global__ __launch_bounds__(256) void migrate_collect_kernel(const int32_t *prio, const int64_t *obj,
                                                              int32_t *stage_prio, int64_t *stage_obj,
                                                              int K, int n, int mig_k) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  migrate_collect_island(prio, obj, stage_prio, stage_obj, blockIdx.x, K, n, mig_k, taken, sv, si);
}

__global__ __launch_bounds__(256) void migrate_apply_kernel(int32_t *prio, int64_t *obj,
                                                            int32_t *elite, int64_t *elite_obj,
                                                            const int32_t *stage_prio,
                                                            const int64_t *stage_obj, int K, int n,
                                                            int mig_k, int islands) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  migrate_apply_island(prio, obj, elite, elite_obj, stage_prio, stage_obj, blockIdx.x, K, n, mig_k,
                       islands, taken, sv, si);
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
// Batched GA: slots of independent instances advanced by the same launches.
// ---------------------------------------------------------------------------
struct BatchSlot {
  DInst I;              // pq points into the slot's region of the workspace
  int32_t *prio[2];     // generation g lives in prio[g & 1]
  int64_t *obj[2];
  int32_t *elite;
  int64_t *elite_obj;
  int32_t *stage_prio;
  int64_t *stage_obj;
  u64 seed, shop;
  int32_t event;
  int32_t gen;          // generations run since the slot was set (advanced on the device)
  int32_t active;
  int32_t cap;          // on-chip profile slots of this slot's decodes
  int32_t cls;          // profile size class: the generation launch that decodes this slot
  int32_t span;         // longest schedule (end - RS) of generation 0
};

struct BatchArgs {
  BatchSlot *slots;
  Header *hdr;
  uint8_t *gprof;       // per persistent block: an off-chip profile of gstride bytes
  size_t gstride;
  int32_t n_slots, pop, rows, cols, islands, mig_k, mig_interval;
  uint32_t pc, pm;
};

// Read a struct the kernel never writes through the scalar cache, word by word.
template <class T>
__device__ __forceinline__ T ld_const_struct(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  typedef __attribute__((address_space(4))) const uint32_t cw;
  T out;
  const cw *src = (const cw *)p;
  uint32_t *dst = (uint32_t *)&out;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) dst[k] = src[k];
  return out;
}

__device__ __forceinline__ GaDev slot_ga(const BatchSlot &S, const BatchArgs &B, int gen) {
  GaDev A;
  A.prio_in = S.prio[(gen - 1) & 1];
  A.obj_in = S.obj[(gen - 1) & 1];
  A.prio_out = S.prio[gen & 1];
  A.obj_out = S.obj[gen & 1];
  A.elite = S.elite;
  A.elite_obj = S.elite_obj;
  A.stage_prio = S.stage_prio;
  A.stage_obj = S.stage_obj;
  A.hdr = B.hdr;
  A.ovf_list = nullptr;
  A.redo_prof = nullptr;
  A.redo_stride = 0;
  A.seed = S.seed;
  A.shop = S.shop;
  A.event = S.event;
  A.rows = B.rows;
  A.cols = B.cols;
  A.islands = B.islands;
  A.isl0 = 0;
  A.narrow = 0;
  A.mig_k = B.mig_k;
  A.pc = B.pc;
  A.pm = B.pm;
  return A;
}

// Decode the child in l.gene (already stored in A.prio_out) with the on-chip
// profile; a decode that outgrows it is redone at once with this block's
// off-chip profile.
template <int MAXM>
__device__ void decode_slot(const DInst &I, const GaDev &A, int i, int cap, const Lds &l,
                            const GlobalProfile &gp, int32_t *span_max = nullptr) {
  int64_t work = 0;
  int st = decode_core<MAXM, false>(I, l, LdsProfile{l.prof, cap}, A.obj_out + i, &work, nullptr,
                                    nullptr, span_max);
  if (st == kDecOverflow) {
    const int32_t *src = A.prio_out + (size_t)i * I.n;
    for (int k = __lane_id(); k < I.n; k += kWave) l.gene[k] = src[k];
    __asm__ volatile("" ::: "memory");
    work = 0;
    st = decode_core<MAXM, false>(I, l, gp, A.obj_out + i, &work, nullptr, nullptr, span_max);
  }
  if (st == kDecOk) {
    if (__lane_id() == 0) atomicAdd(&A.hdr->work, (unsigned long long)work);
    return;
  }
  if (__lane_id() == 0) A.obj_out[i] = -1;
  flag_error(A.hdr, st == kDecOverflow ? kDecInval : st);
}

// (value, index) argmin / argmax over one wave, lowest index on ties.
// One generation of every active slot. ISLAND: an item is an island (its
// slots in turn, then its replacement); otherwise an item is one child.
template <int MAXM, bool ISLAND>
__global__ __launch_bounds__(64) void batch_generation_kernel(BatchArgs B, int cls) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int K = B.rows * B.cols;
  const int per_slot = ISLAND ? B.islands : B.pop;
  const int total = B.n_slots * per_slot;
  uint8_t *gp_mem = B.gprof + B.gstride * blockIdx.x;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    const int d = item / per_slot;
    const BatchSlot S = ld_const_struct(B.slots + d);
    if (!S.active || S.cls != cls) continue;
    const int gen = S.gen + 1;
    const GaDev A = slot_ga(S, B, gen);
    const Lds l = carve_lds(smem, S.I.n);
    const GlobalProfile gp{gp_mem, offchip_cap(S.I.horizon)};
    if (ISLAND) {
      const int isl = item % per_slot;
      for (int k = 0; k < K; ++k) {
        breed_child(A, S.I.n, isl * K + k, gen, l);
        decode_slot<MAXM>(S.I, A, isl * K + k, S.cap, l, gp);
      }
      replace_island_wave(A, isl, K, S.I.n);
    } else {
      const int i = item % per_slot;
      breed_child(A, S.I.n, i, gen, l);
      decode_slot<MAXM>(S.I, A, i, S.cap, l, gp);
    }
  }
}

// Generation 0 of slot d.
template <int MAXM>
__global__ __launch_bounds__(64) void batch_init_kernel(BatchArgs B, int d) {
  extern __shared__ __align__(16) uint8_t smem[];
  const BatchSlot S = ld_const_struct(B.slots + d);
  const GaDev A = slot_ga(S, B, 1);  // generation 0 goes to prio[0]: the "input" side of 1
  GaDev A0 = A;
  A0.prio_out = S.prio[0];
  A0.obj_out = S.obj[0];
  const Lds l = carve_lds(smem, S.I.n);
  const GlobalProfile gp{B.gprof + B.gstride * blockIdx.x, offchip_cap(S.I.horizon)};
  for (int i = blockIdx.x; i < B.pop; i += gridDim.x) {
    init_child(A0, S.I.n, i, l);
    decode_slot<MAXM>(S.I, A0, i, S.cap, l, gp, &B.slots[d].span);
  }
}

// Profile size class of slot d from its generation 0: the smallest of
// caps[0..n_cls) that holds 5/4 of the longest schedule plus 64 slots (the
// largest otherwise), no more than the slot's horizon needs.
__global__ __launch_bounds__(64) void batch_class_kernel(BatchArgs B, int d, int n_cls, int top) {
  if (threadIdx.x != 0) return;
  BatchSlot *S = B.slots + d;
  const int need = S->span + S->span / 4 + 64;
  int c = 0, cap = top >> (n_cls - 1);
  while (c + 1 < n_cls && cap < need) {
    ++c;
    cap <<= 1;
  }
  const int h = (S->I.horizon + 63) / 64 * 64;
  S->cls = c;
  S->cap = cap < h ? cap : h;
}

__global__ __launch_bounds__(256) void batch_replace_kernel(BatchArgs B) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  const int d = blockIdx.x / B.islands, I = blockIdx.x % B.islands;
  const BatchSlot S = ld_const_struct(B.slots + d);
  if (!S.active) return;
  const int cur = (S.gen + 1) & 1;
  replace_island(S.prio[cur], S.obj[cur], S.elite, S.elite_obj, I, B.rows * B.cols, S.I.n, sv, si);
}

__device__ __forceinline__ bool migrates(const BatchArgs &B, int gen) {
  return B.mig_interval > 0 && B.mig_k > 0 && B.islands > 1 && gen % B.mig_interval == 0;
}

__global__ __launch_bounds__(256) void batch_migrate_collect_kernel(BatchArgs B) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  const int d = blockIdx.x / B.islands, I = blockIdx.x % B.islands;
  const BatchSlot S = ld_const_struct(B.slots + d);
  if (!S.active || !migrates(B, S.gen + 1)) return;
  const int cur = (S.gen + 1) & 1;
  migrate_collect_island(S.prio[cur], S.obj[cur], S.stage_prio, S.stage_obj, I, B.rows * B.cols,
                         S.I.n, B.mig_k, taken, sv, si);
}

__global__ __launch_bounds__(256) void batch_migrate_apply_kernel(BatchArgs B) {
  __shared__ int64_t sv[256];
  __shared__ int si[256];
  extern __shared__ uint8_t taken[];
  const int d = blockIdx.x / B.islands, I = blockIdx.x % B.islands;
  const BatchSlot S = ld_const_struct(B.slots + d);
  if (!S.active || !migrates(B, S.gen + 1)) return;
  const int cur = (S.gen + 1) & 1;
  migrate_apply_island(S.prio[cur], S.obj[cur], S.elite, S.elite_obj, S.stage_prio, S.stage_obj, I,
                       B.rows * B.cols, S.I.n, B.mig_k, B.islands, taken, sv, si);
}

// End of a generation: every active slot has one more.
__global__ __launch_bounds__(256) void batch_advance_kernel(BatchArgs B) {
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < B.n_slots; d += gridDim.x * blockDim.x)
    if (B.slots[d].active) B.slots[d].gen += 1;
}

// ---------------------------------------------------------------------------
// Instance preparation: packing, checks, horizon bound, rescheduling.
// ---------------------------------------------------------------------------
// Zero a workspace header with one wave (a kernel, not a memset, so the
// no-allocation decode holds kernels only).
__global__ __launch_bounds__(64) void clear_header_kernel(Header *h) {
  static_assert(kHeaderBytes == 4 * kWave, "one word per lane");
  ((int32_t *)h)[threadIdx.x] = 0;
}

// The decoders' per-instance table: row k * g + s holds stage s of active job
// k (gene order) as P | Q << 16 per machine, omp words (zero past o_max); the
// n words after the rows hold the active jobs' due dates.
__global__ void pack_kernel(const int32_t *proc, const int32_t *power, const int32_t *due,
                            const int32_t *active, uint32_t *pq, int n, int g, int om, int omp) {
  const size_t total = (size_t)n * g * omp;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += step) {
    const size_t row = x / omp;
    const int m = (int)(x % omp);
    const size_t k = row / g, st = row % g;
    uint32_t v = 0;
    if (m < om) {
      const size_t src = ((size_t)active[k] * g + st) * om + m;
      v = ((uint32_t)proc[src] & 0xFFFFu) | (((uint32_t)power[src] & 0xFFFFu) << 16);
    }
    pq[x] = v;
  }
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < (size_t)n; k += step)
    pq[total + k] = (uint32_t)due[active[k]];
}

struct PrepArgs {
  const int32_t *nm, *proc, *power, *first, *ready, *mfree, *running, *active;
  int32_t n_jobs, g, om, q_max, rs, nr, n;
  const int32_t *fixed;
  int32_t nf;
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
  int64_t base = a.rs, sum = 0, ops = 0;
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
    ops += a.g - f;
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
  for (int r = threadIdx.x; r < a.nf; r += blockDim.x) {
    const int st = a.fixed[3 * r], end = a.fixed[3 * r + 1], q = a.fixed[3 * r + 2];
    if (st < a.rs || end <= st || q < 1 || q > 65535) err |= kErrInval;
    if (q > a.q_max) err |= kErrInfeasible;
    base = max(base, (int64_t)end);
  }
  int64_t tot_base, tot_sum, tot_unfrozen, tot_ops;
  block_reduce_i64(base, sh, true, tot_base);
  block_reduce_i64(sum, sh, false, tot_sum);
  block_reduce_i64(unfrozen, sh, false, tot_unfrozen);
  block_reduce_i64(ops, sh, false, tot_ops);
  if (err) atomicOr(&h->err, err);
  if (threadIdx.x == 0) {
    if (tot_unfrozen != a.n) atomicOr(&h->err, kErrInval);
    h->horizon = tot_base - a.rs + tot_sum + 1;
    h->n_ops = (int32_t)tot_ops;
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
  // the traditional static approach: every known job frozen whole, its ops not
  // started by rs kept in place (fixed_o, room for fixed_cap triples)
  int32_t static_mode;
  int32_t *fixed_o;
  int32_t fixed_cap;
};

// Predictive-reactive rescheduling (Section 4.1) in one block of 1024
// threads: freeze ops started before rs (eq. (10)); an op running at rs
// (S < rs < S + P, Algorithm 1) keeps its machine and power until it ends.
__global__ __launch_bounds__(1024) void reschedule_kernel(ReschedArgs a, Header *h) {
  __shared__ int64_t sh[1024];
  __shared__ int scan_run[1024], scan_act[1024], scan_fix[1024];
  __shared__ int carry_run, carry_act, carry_fix;
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
    carry_fix = 0;
  }
  __syncthreads();
  int err = 0;
  int64_t tard = 0, cmax = 0;
  for (int b0 = 0; b0 < n; b0 += T) {
    const int j = b0 + t;
    int run = 0, act = 0, run_end = 0, run_q = 0, nfix = 0;
    if (j < a.n0 && a.static_mode) {
      // Static approach: the job's whole plan stays; each stage's planned
      // completion (kept in column 0 of machine_free) bounds the arrivals.
      int last_end = a.release[j];
      for (int s = 0; s < g; ++s) {
        const int m = a.plan_mach[(size_t)j * g + s], st = a.plan_start[(size_t)j * g + s];
        if (m < 0 || m >= a.nm[s] || st < 0) {
          err |= kErrInval;
          break;
        }
        const int end = st + a.proc[((size_t)j * g + s) * om + m];
        atomicMax(&a.mfree_o[s * om], end);
        if (st < a.rs && end > a.rs) {
          err |= run ? kErrInval : 0;  // two ops of one job running at once
          run = 1;
          run_end = end;
          run_q = a.power[((size_t)j * g + s) * om + m];
        } else if (st >= a.rs) {
          ++nfix;
        }
        last_end = end;
      }
      a.first_o[j] = g;
      a.ready_o[j] = last_end;
      tard += max(last_end - a.due[j], 0);
      cmax = max(cmax, (int64_t)last_end);
    } else if (j < a.n0) {
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
    // ordered compaction of running ops, fixed ops and active jobs (ascending job id)
    scan_run[t] = run;
    scan_act[t] = act;
    scan_fix[t] = nfix;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {
      const int vr = t >= d ? scan_run[t - d] : 0, va = t >= d ? scan_act[t - d] : 0;
      const int vf = t >= d ? scan_fix[t - d] : 0;
      __syncthreads();
      scan_run[t] += vr;
      scan_act[t] += va;
      scan_fix[t] += vf;
      __syncthreads();
    }
    if (nfix) {
      int pos = carry_fix + scan_fix[t] - nfix;
      for (int s = 0; s < g; ++s) {
        const int m = a.plan_mach[(size_t)j * g + s], st = a.plan_start[(size_t)j * g + s];
        if (st < a.rs) continue;
        if (pos >= a.fixed_cap) {
          err |= kErrInval;
          break;
        }
        a.fixed_o[3 * pos] = st;
        a.fixed_o[3 * pos + 1] = st + a.proc[((size_t)j * g + s) * om + m];
        a.fixed_o[3 * pos + 2] = a.power[((size_t)j * g + s) * om + m];
        ++pos;
      }
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
      carry_fix += scan_fix[t];
    }
    __syncthreads();
  }
  if (a.static_mode)  // every machine of a stage is free from the stage's planned completion
    for (int x = t; x < g * om; x += T)
      if (x % om) a.mfree_o[x] = x % om < a.nm[x / om] ? a.mfree_o[x - x % om] : 0;
  int64_t tot_tard, tot_cmax;
  block_reduce_i64(tard, sh, false, tot_tard);
  block_reduce_i64(cmax, sh, true, tot_cmax);
  if (err) atomicOr(&h->err, err);
  if (t == 0) {
    h->frozen_tardiness = tot_tard;
    h->frozen_cmax = (int32_t)tot_cmax;
    h->n_running = carry_run;
    h->n_active = carry_act;
    h->n_fixed = a.static_mode ? min(carry_fix, a.fixed_cap) : 0;
  }
  __threadfence_block();
  __syncthreads();
  PrepArgs p{a.nm, a.proc_o, a.power_o, a.first_o, a.ready_o, a.mfree_o, a.running_o, a.active_o,
             n, g, om, a.q_max, a.rs, min(carry_run, a.running_cap), carry_act,
             a.static_mode ? a.fixed_o : nullptr, a.static_mode ? min(carry_fix, a.fixed_cap) : 0};
  prepare_body(p, h);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------
constexpr int kTimingFamilies = 7;
constexpr int kTimingStep = 6;  // ga_step spans, counted in generations
struct Timing {
  std::mutex mu;
  bool on = false;
  uint32_t mask = 0;  // bit f: family f is timed
  int32_t every = 1;  // one launch in `every` of a timed family gets events
  int64_t seen[kTimingFamilies] = {};
  std::vector<hipEvent_t> ev[kTimingFamilies];
  size_t used[kTimingFamilies] = {};
  double ms[kTimingFamilies] = {};
  int64_t launches[kTimingFamilies] = {};
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
  if (family >= 0 && g_timing.on && ((g_timing.mask >> family) & 1u) &&
      g_timing.seen[family]++ % g_timing.every == 0) {
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

// Events around a whole ga_step call on the caller's stream (kTimingStep): the
// span from before its first launch to after its island groups are joined.
// Returns the event pair's index, or -1 when the family is not timed.
int span_begin(hipStream_t s) {
  if (!g_timing.on || !((g_timing.mask >> kTimingStep) & 1u)) return -1;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (g_timing.used[kTimingStep] == kTimingPairs) {
    drain_family(kTimingStep, kTimingPairs);
    g_timing.used[kTimingStep] = 0;
  }
  const int k = (int)g_timing.used[kTimingStep]++;
  (void)hipEventRecord(g_timing.ev[kTimingStep][2 * k], s);
  return k;
}
void span_end(int k, hipStream_t s, int64_t generations) {
  if (k < 0) return;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  (void)hipEventRecord(g_timing.ev[kTimingStep][2 * k + 1], s);
  g_timing.launches[kTimingStep] += generations;
}

int max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

int omp_of(int om) { return om <= 4 ? 4 : om <= 8 ? 8 : 16; }

int check_host(const ffs_instance *in) {
  if (!in) return FFS_E_INVAL;
  if (in->n_stages < 1 || in->o_max < 1 || in->n_jobs < 0 || in->n_active < 0 ||
      in->n_active > in->n_jobs || in->n_running < 0 || in->q_max < 1 || in->n_fixed < 0)
    return FFS_E_INVAL;
  if (in->o_max > 16 || in->n_stages > kMaxStages || in->n_jobs >= (1 << 20) || in->q_max > 255 ||
      in->n_active > kMaxGenes || in->rs < 0 || in->rs >= kMaxTime)
    return FFS_E_UNSUPPORTED;
  if (!in->n_machines || !in->proc || !in->power || !in->due || !in->first_stage || !in->ready ||
      !in->machine_free || (in->n_running && !in->running) || (in->n_active && !in->active) ||
      (in->n_fixed && !in->fixed))
    return FFS_E_INVAL;
  return FFS_OK;
}

// pq: the table pack_kernel wrote at row width omp (0: omp_of(o_max)).
DInst make_dinst(const ffs_instance *in, const uint32_t *pq, int omp = 0) {
  DInst d;
  if (omp == 0) omp = omp_of(in->o_max);
  d.pq = pq;
  d.due_k = (const int32_t *)(pq + (size_t)in->n_active * in->n_stages * omp);
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
  d.omp = omp;
  d.q_max = in->q_max;
  d.wt = in->wt;
  d.rs = in->rs;
  d.nr = in->n_running;
  d.fixed = in->fixed;
  d.nf = in->n_fixed;
  d.n = in->n_active;
  d.frozen_cmax = in->frozen_cmax;
  d.horizon = in->horizon;
  d.rules = in->decode_rules;
  return d;
}

int resolve_cap(const ffs_instance *in, int32_t lds_slots) {
  int cap = lds_slots > 0 ? lds_slots : kDefaultLdsSlots;
  const int64_t h = align_up((size_t)in->horizon, 64);
  if (cap > h) cap = (int)h;
  cap = (int)align_up((size_t)(cap < 64 ? 64 : cap), 64);
  return cap;
}

// Bytes of pack_kernel's table: n x g rows of omp words, then n due dates.
size_t pq_bytes(int n, int g, int omp) {
  return align_up((size_t)n * g * omp * 4 + (size_t)n * 4 + 64, 256);
}
size_t pq_bytes(const ffs_instance *in) {
  return pq_bytes(in->n_active, in->n_stages, omp_of(in->o_max));
}

struct DecodeLayout {
  Header *hdr;
  uint32_t *pq;
  int32_t *xyop, *xyg0;  // X/Y gene table (ffs_decode_xy)
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
  L.xyop = (int32_t *)(b + off);
  off += align_up((size_t)4 * in->n_ops + 4, 256);
  L.xyg0 = (int32_t *)(b + off);
  off += align_up((size_t)4 * in->n_active + 4, 256);
  if (cap < in->horizon) {
    L.ovf_list = (int32_t *)(b + off);
    off += align_up((size_t)pop * 4, 256);
    L.gstride = align_up((size_t)offchip_cap(in->horizon) + 64, 256);
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
               L.gstride, (int32_t *)nullptr);
    if (e != hipSuccess) return FFS_E_DEVICE;
  }
  return FFS_OK;
}

template <int MAXM>
int run_decode_xy(const ffs_instance *in, const int32_t *genes, int32_t pop, int64_t *obj,
                  int32_t *start, int32_t *mach, int64_t *work, int cap, const DecodeLayout &L,
                  hipStream_t stream) {
  const DInst d = make_dinst(in, L.pq);
  const XyTab T{L.xyop, L.xyg0, in->n_ops};
  const size_t shmem = lds_bytes_xy(in->n_active, in->n_ops, in->n_stages, in->o_max, cap);
  hipError_t e = launch(0, decode_xy_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, T,
                        genes, obj, work, start, mach, L.hdr, L.ovf_list, cap);
  if (e != hipSuccess) return FFS_E_DEVICE;
  if (cap < in->horizon) {
    e = launch(3, overflow_xy_kernel<MAXM>, dim3(kFixBlocks), dim3(kWave),
               lds_bytes_xy(in->n_active, in->n_ops, in->n_stages, in->o_max, 0), stream, d, T,
               genes, obj, work, start, mach, L.hdr, (const int32_t *)L.ovf_list, L.gprof,
               L.gstride);
    if (e != hipSuccess) return FFS_E_DEVICE;
  }
  return FFS_OK;
}

int build_xy_table(const ffs_instance *in, int32_t *op, int32_t *g0, hipStream_t stream);

int pack(const ffs_instance *in, uint32_t *pq, hipStream_t stream, int omp = 0) {
  if (in->n_active == 0) return FFS_OK;
  if (omp == 0) omp = omp_of(in->o_max);
  const size_t words = (size_t)in->n_active * in->n_stages * omp;
  const int blocks = (int)((words + 255) / 256);
  hipError_t e = launch(-1, pack_kernel, dim3(blocks < 1024 ? blocks : 1024), dim3(256), 0, stream,
                        in->proc, in->power, in->due, in->active, pq, in->n_active,
                        in->n_stages, in->o_max, omp);
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
  int32_t *xyop, *xyg0;  // X/Y gene table (encoding 1)
  u64 *prefix;           // running fitness sums (FFS_GA_CLASSICAL)
  uint8_t *gprof;
  size_t gstride, total;
  bool inline_redo;  // one off-chip profile per individual: no overflow kernel
};

// Genes per chromosome: one priority per active job, or X and Y (2R).
int64_t chrom_len(const ffs_instance *in, const ffs_ga_params *p) {
  return p->encoding == 1 ? 2 * (int64_t)in->n_ops : (int64_t)in->n_active;
}

// Off-chip profiles of one per individual are used up to this many bytes;
// past it the overflow kernel redoes overflowed decodes with kFixBlocks of them.
constexpr size_t kInlineRedoBytes = (size_t)1 << 30;

GaLayout ga_layout(void *ws, const ffs_instance *in, const ffs_ga_params *p, int cap) {
  GaLayout L{};
  uint8_t *b = (uint8_t *)ws;
  const size_t pop = (size_t)p->islands * p->rows * p->cols, n = (size_t)chrom_len(in, p);
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
  if (p->scheme == FFS_GA_CLASSICAL) {
    L.prefix = (u64 *)(b + off);
    off += align_up(pop * 8, 256);
  }
  if (p->encoding == 1) {
    L.xyop = (int32_t *)(b + off);
    off += align_up((size_t)4 * in->n_ops + 4, 256);
    L.xyg0 = (int32_t *)(b + off);
    off += align_up((size_t)4 * in->n_active + 4, 256);
  }
  if (cap < in->horizon) {
    L.gstride = align_up((size_t)offchip_cap(in->horizon) + 64, 256);
    L.gprof = b + off;
    L.inline_redo = pop * L.gstride <= kInlineRedoBytes;
    off += (L.inline_redo ? pop : (size_t)kFixBlocks) * L.gstride;
  }
  L.total = off;
  return L;
}

// The on-chip slots a GA workspace layout is computed with: with FFS_LDS_AUTO
// the slots are only known after generation 0, so the layout always holds the
// off-chip profiles.
int layout_cap(const ffs_ga_params *p, int cap) { return p->lds_slots == FFS_LDS_AUTO ? 0 : cap; }

// On-chip slots FFS_LDS_AUTO works with: as many as one workgroup's LDS holds
// next to the chromosome's arrays, at most `limit` and no more than the horizon
// needs. The sizing decode of generation 0 keeps at most kProbeSlots (a longer
// schedule is decoded again off chip, which records its length too, and the
// smaller allocation lets more of its waves run at once); later generations may
// keep up to kAutoSlots.
constexpr int64_t kProbeSlots = 16384, kAutoSlots = 32768;
int probe_cap(const ffs_instance *in, int64_t limit = kProbeSlots) {
  const int64_t h = (int64_t)align_up((size_t)in->horizon, 64);
  const int64_t room = (int64_t)max_lds_bytes() - (int64_t)lds_head(in->n_active) - kWave;
  int64_t cap = room / 64 * 64;
  if (cap > limit) cap = limit;
  if (cap > h) cap = h;
  return (int)(cap < 64 ? 64 : cap);
}

int check_ga_params(const ffs_ga_params *p) {
  if (!p || p->islands < 1 || p->rows < 1 || p->cols < 1 || p->mig_k < 0 || p->mig_interval < 0)
    return FFS_E_INVAL;
  const int64_t K = (int64_t)p->rows * p->cols;
  if (p->mig_k > K) return FFS_E_INVAL;
  if (K > 65536 || K * p->islands > (1 << 26)) return FFS_E_UNSUPPORTED;
  if (p->encoding != 0 && p->encoding != 1) return FFS_E_INVAL;
  if (p->scheme != FFS_GA_HYBRID && p->scheme != FFS_GA_CLASSICAL && p->scheme != FFS_GA_CELLULAR)
    return FFS_E_INVAL;
  if (p->scheme != FFS_GA_HYBRID && (p->islands != 1 || p->encoding != 0)) return FFS_E_INVAL;
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
  A.redo_prof = L.inline_redo ? L.gprof : nullptr;
  A.redo_stride = L.gstride;
  A.seed = ga->seed;
  A.shop = ga->shop;
  A.event = ga->event;
  A.rows = ga->params.rows;
  A.cols = ga->params.cols;
  A.islands = ga->params.islands;
  A.isl0 = 0;
  A.narrow = 0;
  A.mig_k = ga->params.mig_k;
  A.pc = ga->params.pc;
  A.pm = ga->params.pm;
  return A;
}

template <int MAXM>
int ga_overflow(const ffs_instance *in, const GaLayout &L, int buf, int cap, hipStream_t stream,
                bool xy = false, int32_t *span = nullptr) {
  if (cap >= in->horizon || L.inline_redo) return FFS_OK;
  const DInst d = make_dinst(in, L.pq);
  hipError_t e;
  if (xy)
    e = launch(3, overflow_xy_kernel<MAXM>, dim3(kFixBlocks), dim3(kWave),
               lds_bytes_xy(in->n_active, in->n_ops, in->n_stages, in->o_max, 0), stream, d,
               XyTab{L.xyop, L.xyg0, in->n_ops}, (const int32_t *)L.prio[buf], L.obj[buf],
               (int64_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, L.hdr,
               (const int32_t *)L.ovf_list, L.gprof, L.gstride);
  else
    e = launch(3, overflow_kernel<MAXM>, dim3(kFixBlocks), dim3(kWave),
               lds_bytes(in->n_active, 0), stream, d, (const int32_t *)L.prio[buf],
               L.obj[buf], (int64_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, L.hdr,
               (const int32_t *)L.ovf_list, L.gprof, L.gstride, span);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

int build_xy_table(const ffs_instance *in, int32_t *op, int32_t *g0, hipStream_t stream) {
  return launch(-1, xy_table_kernel, dim3(1), dim3(1024), 0, stream, in->first_stage, in->active,
                in->n_machines, in->n_active, in->n_stages, op, g0) == hipSuccess
             ? FFS_OK
             : FFS_E_DEVICE;
}

// Single-wave workgroups of the generation kernel that one compute unit holds at
// `bytes` of LDS each (the runtime's occupancy figure: LDS granularity,
// registers and wave slots included); 0 if the runtime cannot say.
template <int MAXM>
int waves_per_cu(size_t bytes) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void *)ga_generation_kernel<MAXM>,
                                                   kWave, bytes) != hipSuccess)
    return 0;
  return b;
}

int n_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return v;
}

// Whether the generation and init kernels take the narrow layout: under the
// default rules, and only where it lets a compute unit hold more waves of a
// population that the chip cannot hold at once in the wide layout (otherwise
// the narrow form's extra masking buys nothing).
template <int MAXM>
bool use_narrow(const ffs_instance *in, int cap, int pop) {
  if (in->decode_rules != 0) return false;
  const int ww = waves_per_cu<MAXM>(lds_bytes(in->n_active, cap));
  const int wn = waves_per_cu<MAXM>(lds_bytes_n(in->n_active, cap));
  return wn > ww && (int64_t)pop > (int64_t)ww * n_cus();
}

template <int MAXM>
int ga_init_impl(ffs_ga *ga, const ffs_instance *in, const GaLayout &L, hipStream_t stream,
                 bool auto_cap) {
  const DInst d = make_dinst(in, L.pq);
  GaDev A = make_gadev(ga, L, 1);  // generation 0 is written to buffer 0
  const int pop = ga->pop, cap = ga->lds_slots, n = ga->n_genes;
  const int K = ga->params.rows * ga->params.cols;
  const bool xy = ga->params.encoding == 1, hybrid = ga->params.scheme == FFS_GA_HYBRID;
  int rc;
  if (xy) {
    if ((rc = build_xy_table(in, L.xyop, L.xyg0, stream))) return rc;
    if (launch(1, ga_init_xy_kernel, dim3(pop), dim3(kWave),
               lds_bytes_xy(in->n_active, in->n_ops, in->n_stages, in->o_max, cap), stream, d,
               XyTab{L.xyop, L.xyg0, in->n_ops}, A, cap) != hipSuccess)
      return FFS_E_DEVICE;
  } else {
    A.narrow = hybrid && use_narrow<MAXM>(in, cap, pop);
    if (launch(1, ga_init_kernel<MAXM>, dim3(pop), dim3(kWave), lds_bytes_gen(in, cap, A.narrow),
               stream, d, A, cap, auto_cap ? &L.hdr->span_max : (int32_t *)nullptr) != hipSuccess)
      return FFS_E_DEVICE;
  }
  rc = ga_overflow<MAXM>(in, L, 0, cap, stream, xy, auto_cap ? &L.hdr->span_max : nullptr);
  if (rc) return rc;
  if (launch(-1, elite_init_kernel, dim3(ga->params.islands), dim3(256), 0, stream,
             (const int32_t *)L.prio[0], (const int64_t *)L.obj[0], L.elite, L.elite_obj, K,
             n) != hipSuccess)
    return FFS_E_DEVICE;
  if (ga->params.scheme == FFS_GA_CLASSICAL &&
      launch(-1, emax_kernel, dim3(1), dim3(256), 0, stream, (const int64_t *)L.obj[0], pop,
             L.hdr) != hipSuccess)
    return FFS_E_DEVICE;
  if (auto_cap) {
    // Later generations: generation 0's longest schedule plus 1/64 and 64 slots,
    // then widened to the most slots (at most kAutoSlots) that keep as many waves
    // per compute unit.
    Header host;
    if ((rc = read_header(L.hdr, &host, stream))) return rc;
    const int64_t span = host.span_max, top = probe_cap(in, kAutoSlots);
    int64_t lo = (int64_t)align_up((size_t)(span + span / 64 + 64), 64);
    if (lo > top) lo = top;
    // the layout the generations will take at lo sets the bytes per slot count
    const bool narrow = hybrid && use_narrow<MAXM>(in, (int)lo, pop);
    const int w = waves_per_cu<MAXM>(lds_bytes_gen(in, (int)lo, narrow));
    int64_t a = lo / 64, b = top / 64;  // waves_per_cu falls as the slots grow
    while (w > 0 && a < b) {
      const int64_t m = (a + b + 1) / 2;
      if (waves_per_cu<MAXM>(lds_bytes_gen(in, (int)(m * 64), narrow)) >= w)
        a = m;
      else
        b = m - 1;
    }
    ga->lds_slots = (int32_t)(a * 64);
  }
  return FFS_OK;
}

constexpr int kMaxDevices = 64;

// Island groups of ga_step. Between two migrations the islands of a GA share
// nothing, so ga_step can run groups of islands on streams of their own: a group
// that has decoded its slowest chromosome and replaced its islands starts its
// next generation while the other groups still decode, and the compute units
// stay busy through each launch's tail instead of waiting at a barrier over the
// whole population. Every draw is keyed by the global slot, so the results do
// not depend on the grouping. Group 0 runs on the caller's stream; groups 1..
// run on per-device streams of this library (default priority, not blocking
// the null stream), forked from and joined back into the caller's stream with
// events, before and after every migration and at the end of the call.
constexpr int kMaxGroups = 4;
std::atomic<int> g_island_groups{0};  // 0: automatic (kMaxGroups)

struct GroupStreams {
  hipStream_t s[kMaxGroups] = {};  // s[0] stays null: group 0 is the caller's stream
  hipEvent_t fork = nullptr, join[kMaxGroups] = {};
  bool ready = false;
};
// Held across a grouped ga_step's launches: two host threads would otherwise
// re-record one fork or join event between another's record and wait.
std::mutex g_group_mu;
GroupStreams g_groups[kMaxDevices];

void release_groups(GroupStreams &G) {
  for (int g = 1; g < kMaxGroups; ++g) {
    if (G.s[g]) (void)hipStreamDestroy(G.s[g]);
    if (G.join[g]) (void)hipEventDestroy(G.join[g]);
    G.s[g] = nullptr;
    G.join[g] = nullptr;
  }
  if (G.fork) (void)hipEventDestroy(G.fork);
  G.fork = nullptr;
}

// This device's group streams and events, created on first use (the caller
// holds g_group_mu).
int group_streams(GroupStreams **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FFS_E_DEVICE;
  GroupStreams &G = g_groups[dev];
  if (!G.ready) {
    bool ok = hipEventCreateWithFlags(&G.fork, hipEventDisableTiming) == hipSuccess;
    for (int g = 1; ok && g < kMaxGroups; ++g)
      ok = hipStreamCreateWithFlags(&G.s[g], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&G.join[g], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      release_groups(G);
      return FFS_E_DEVICE;
    }
    G.ready = true;
  }
  *out = &G;
  return FFS_OK;
}

// A screened generation's surrogate inputs (ffs_surrogate.h).
struct Screen {
  const float *table, *theta;
  int variants;
  float *scores;
  int32_t *choice;
};

bool migrates(const ffs_ga_params &p, int gen) {
  return p.mig_interval > 0 && p.mig_k > 0 && p.islands > 1 && gen % p.mig_interval == 0;
}

// Ring migration after the generation written to buffer 1 - cur.
bool migrate(const ffs_ga_params &p, const GaLayout &L, int cur, int n, hipStream_t stream) {
  const int K = p.rows * p.cols;
  return launch(-1, migrate_collect_kernel, dim3(p.islands), dim3(256), (size_t)K, stream,
                (const int32_t *)L.prio[1 - cur], (const int64_t *)L.obj[1 - cur], L.stage_prio,
                L.stage_obj, K, n, p.mig_k) == hipSuccess &&
         launch(-1, migrate_apply_kernel, dim3(p.islands), dim3(256), (size_t)K, stream,
                L.prio[1 - cur], L.obj[1 - cur], L.elite, L.elite_obj,
                (const int32_t *)L.stage_prio, (const int64_t *)L.stage_obj, K, n, p.mig_k,
                p.islands) == hipSuccess;
}

// ga_step of the hybrid GA over G > 1 island groups (GroupStreams): group g
// holds islands [islands * g / G, islands * (g + 1) / G).
template <int MAXM>
int ga_step_groups(ffs_ga *ga, const ffs_instance *in, const GaLayout &L, int32_t n_gen,
                   hipStream_t stream, int G, size_t shmem, const Screen *scr, bool narrow) {
  std::lock_guard<std::mutex> lk(g_group_mu);
  GroupStreams *GS = nullptr;
  int rc = group_streams(&GS);
  if (rc) return rc;
  const ffs_ga_params &p = ga->params;
  const DInst d = make_dinst(in, L.pq);
  const int K = p.rows * p.cols, n = ga->n_genes, cap = ga->lds_slots;
  const bool xy = p.encoding == 1;
  const XyTab T{L.xyop, L.xyg0, in->n_ops};
  bool ok = true, forked = false;
  auto join = [&]() {
    for (int g = 1; g < G; ++g)
      ok = hipEventRecord(GS->join[g], GS->s[g]) == hipSuccess &&
           hipStreamWaitEvent(stream, GS->join[g], 0) == hipSuccess && ok;
    forked = false;
  };
  for (int32_t k = 0; ok && k < n_gen; ++k) {
    const int gen = ga->generation + 1, cur = ga->cur;
    if (!forked) {
      forked = true;
      ok = hipEventRecord(GS->fork, stream) == hipSuccess;
      for (int g = 1; ok && g < G; ++g)
        ok = hipStreamWaitEvent(GS->s[g], GS->fork, 0) == hipSuccess;
    }
    for (int g = 0; ok && g < G; ++g) {
      const hipStream_t sg = g ? GS->s[g] : stream;
      const int i0 = (int)((int64_t)p.islands * g / G);
      const int i1 = (int)((int64_t)p.islands * (g + 1) / G);
      GaDev A = make_gadev(ga, L, cur);
      A.isl0 = i0;
      A.islands = i1 - i0;
      A.narrow = narrow;
      const dim3 grid((unsigned)((i1 - i0) * K));
      const hipError_t e =
          scr ? launch(5, ga_screened_kernel<MAXM>, grid, dim3(kWave), shmem, sg, d, A, gen, cap,
                       scr->table, scr->theta, scr->variants, scr->scores, scr->choice, ga->pop)
          : xy ? launch(1, ga_generation_xy_kernel, grid, dim3(kWave), shmem, sg, d, T, A, gen, cap)
               : launch(1, ga_generation_kernel<MAXM>, grid, dim3(kWave), shmem, sg, d, A, gen, cap);
      ok = e == hipSuccess &&
           launch(2, replace_wave_kernel, dim3(i1 - i0), dim3(kWave), 0, sg,
                  L.prio[1 - cur] + (size_t)i0 * K * n, L.obj[1 - cur] + (size_t)i0 * K,
                  L.elite + (size_t)i0 * n, L.elite_obj + i0, K, n) == hipSuccess;
    }
    if (ok && migrates(p, gen)) {
      join();
      ok = ok && migrate(p, L, cur, n, stream);
    }
    if (ok) {
      ga->cur = 1 - cur;
      ga->generation = gen;
    }
  }
  if (forked) join();
  return ok ? FFS_OK : FFS_E_DEVICE;
}

template <int MAXM>
int ga_step_impl(ffs_ga *ga, const ffs_instance *in, int32_t n_gen, hipStream_t stream,
                 const Screen *scr = nullptr) {
  GaLayout L = ga_layout(ga->workspace, in, &ga->params, layout_cap(&ga->params, ga->lds_slots));
  const DInst d = make_dinst(in, L.pq);
  const int pop = ga->pop, cap = ga->lds_slots, n = ga->n_genes;
  const int K = ga->params.rows * ga->params.cols;
  const bool xy = ga->params.encoding == 1;
  const XyTab T{L.xyop, L.xyg0, in->n_ops};
  // shmem: the screened and comparison kernels; shmem_gen: the generation kernel
  const size_t shmem = xy ? lds_bytes_xy(in->n_active, in->n_ops, in->n_stages, in->o_max, cap)
                          : lds_bytes(in->n_active, cap);
  const bool narrow = !xy && ga->params.scheme == FFS_GA_HYBRID && use_narrow<MAXM>(in, cap, pop);
  const size_t shmem_gen = xy ? shmem : lds_bytes_gen(in, cap, narrow);
  ga->narrow_lds = narrow && !scr;
  // Island groups for the hybrid GA whose overflowed decodes are redone by their
  // own waves (the overflow kernel's list belongs to the whole population).
  if (ga->params.scheme == FFS_GA_HYBRID && (cap >= in->horizon || L.inline_redo)) {
    const int want = g_island_groups.load();
    int G = want > 0 ? want : kMaxGroups;
    if (G > ga->params.islands) G = ga->params.islands;
    if (G > 1) {
      ga->island_groups = G;
      return ga_step_groups<MAXM>(ga, in, L, n_gen, stream, G, scr ? shmem : shmem_gen, scr,
                                  narrow && !scr);
    }
  }
  ga->island_groups = 1;
  for (int32_t k = 0; k < n_gen; ++k) {
    const int gen = ga->generation + 1;
    const int cur = ga->cur;
    GaDev A = make_gadev(ga, L, cur);
    A.narrow = narrow;
    hipError_t e;
    const int32_t scheme = ga->params.scheme;
    if (scheme == FFS_GA_CLASSICAL) {
      if (launch(-1, fitness_scan_kernel, dim3(1), dim3(1024), 0, stream,
                 (const int64_t *)A.obj_in, pop, (const Header *)L.hdr, L.prefix) != hipSuccess)
        return FFS_E_DEVICE;
      e = launch(1, classical_generation_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, A,
                 gen, cap, (const u64 *)L.prefix);
    } else if (scheme == FFS_GA_CELLULAR) {
      e = launch(1, cellular_generation_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, A,
                 gen, cap);
    } else if (scr)
      e = launch(5, ga_screened_kernel<MAXM>, dim3(pop), dim3(kWave), shmem, stream, d, A, gen, cap,
                 scr->table, scr->theta, scr->variants, scr->scores, scr->choice, pop);
    else if (xy)
      e = launch(1, ga_generation_xy_kernel, dim3(pop), dim3(kWave), shmem, stream, d, T, A, gen,
                 cap);
    else
      e = launch(1, ga_generation_kernel<MAXM>, dim3(pop), dim3(kWave), shmem_gen, stream, d, A,
                 gen, cap);
    if (e != hipSuccess) return FFS_E_DEVICE;
    int rc = ga_overflow<MAXM>(in, L, 1 - cur, cap, stream, xy);
    if (rc) return rc;
    if (scheme == FFS_GA_CELLULAR) {
      if (launch(2, cellular_accept_kernel, dim3(pop), dim3(kWave), 0, stream,
                 (const int32_t *)L.prio[cur], (const int64_t *)L.obj[cur], L.prio[1 - cur],
                 L.obj[1 - cur], n) != hipSuccess ||
          launch(2, elite_update_kernel, dim3(1), dim3(kWave), 0, stream,
                 (const int32_t *)L.prio[1 - cur], (const int64_t *)L.obj[1 - cur], L.elite,
                 L.elite_obj, pop, n) != hipSuccess)
        return FFS_E_DEVICE;
      ga->cur = 1 - cur;
      ga->generation = gen;
      continue;
    }
    if (launch(2, replace_wave_kernel, dim3(ga->params.islands), dim3(kWave), 0, stream,
               L.prio[1 - cur], L.obj[1 - cur], L.elite, L.elite_obj, K, n) != hipSuccess)
      return FFS_E_DEVICE;
    if (migrates(ga->params, gen) && !migrate(ga->params, L, cur, n, stream))
      return FFS_E_DEVICE;
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
  (void)hipFuncSetAttribute((const void *)ga_screened_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)classical_generation_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)cellular_generation_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)decode_xy_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)overflow_xy_kernel<MAXM>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)ga_init_xy_kernel,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)ga_generation_xy_kernel,
                      hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

// ---------------------------------------------------------------------------
// Batched GA host side.
// ---------------------------------------------------------------------------
struct BatchLayout {
  Header *hdr;
  BatchSlot *slots;
  uint8_t *slot_base;
  size_t slot_stride;
  size_t off_pq, off_prio[2], off_obj[2], off_elite, off_eobj, off_sprio, off_sobj;
  uint8_t *gprof;
  size_t gstride, total;
};

int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  return v > 0 ? v : 256;
}

int batch_blocks(const ffs_batch_params *p) { return p->blocks > 0 ? p->blocks : 8 * device_cus(); }

BatchLayout batch_layout(void *ws, const ffs_batch_params *p) {
  BatchLayout L{};
  uint8_t *b = (uint8_t *)ws;
  const size_t pop = (size_t)p->ga.islands * p->ga.rows * p->ga.cols;
  const size_t n = (size_t)p->max_genes, kk = p->ga.mig_k > 0 ? p->ga.mig_k : 1;
  size_t off = 0;
  L.hdr = (Header *)(b + off);
  off += kHeaderBytes;
  L.slots = (BatchSlot *)(b + off);
  off += align_up(sizeof(BatchSlot) * p->n_slots, 256);
  // one slot's region
  size_t so = 0;
  L.off_pq = so;
  so += pq_bytes(p->max_genes, p->max_stages, omp_of(p->o_max));
  for (int k = 0; k < 2; ++k) {
    L.off_prio[k] = so;
    so += align_up(pop * n * 4 + 4, 256);
    L.off_obj[k] = so;
    so += align_up(pop * 8, 256);
  }
  L.off_elite = so;
  so += align_up((size_t)p->ga.islands * n * 4 + 4, 256);
  L.off_eobj = so;
  so += align_up((size_t)p->ga.islands * 8, 256);
  L.off_sprio = so;
  so += align_up((size_t)p->ga.islands * kk * n * 4 + 4, 256);
  L.off_sobj = so;
  so += align_up((size_t)p->ga.islands * kk * 8, 256);
  L.slot_stride = so;
  L.slot_base = b + off;
  off += so * p->n_slots;
  L.gstride = align_up((size_t)offchip_cap(p->max_horizon) + kWave, 256);
  L.gprof = b + off;
  off += L.gstride * batch_blocks(p);
  L.total = off;
  return L;
}

int batch_classes(const ffs_batch_params *p) {
  return p->profile_classes > 1 ? p->profile_classes : 1;
}

int check_batch_params(const ffs_batch_params *p) {
  if (!p || p->n_slots < 1 || p->max_jobs < 1 || p->max_genes < 1 || p->max_stages < 1 ||
      p->o_max < 1 || p->max_horizon < 1 || p->blocks < 0 || p->profile_classes < 0 ||
      p->profile_classes > FFS_BATCH_MAX_CLASSES ||
      (p->schedule != FFS_SCHEDULE_CHROMOSOME && p->schedule != FFS_SCHEDULE_ISLAND))
    return FFS_E_INVAL;
  int rc = check_ga_params(&p->ga);
  if (rc) return rc;
  if (p->ga.encoding != 0 || p->ga.scheme != FFS_GA_HYBRID)
    return FFS_E_UNSUPPORTED;  // batches run the hybrid GA on job-priority chromosomes
  if (p->n_slots > FFS_BATCH_MAX_SLOTS || p->o_max > 16 || p->max_genes > kMaxGenes ||
      p->max_stages > kMaxStages || p->max_jobs >= (1 << 20) || p->max_horizon >= kMaxTime)
    return FFS_E_UNSUPPORTED;
  return FFS_OK;
}

// On-chip profile slots of the largest class: a multiple of 64 << (classes - 1)
// so that every class (cap >> k) is a multiple of 64.
int batch_cap(const ffs_batch_params *p) {
  const size_t unit = (size_t)64 << (batch_classes(p) - 1);
  int cap = p->ga.lds_slots > 0 ? p->ga.lds_slots : kDefaultLdsSlots;
  cap = (int)align_up((size_t)(cap < 64 ? 64 : cap), unit);
  const int h = (int)align_up((size_t)p->max_horizon, unit);
  return cap > h ? h : cap;
}

BatchArgs batch_args(const ffs_batch *b, const BatchLayout &L) {
  BatchArgs B;
  B.slots = L.slots;
  B.hdr = L.hdr;
  B.gprof = L.gprof;
  B.gstride = L.gstride;
  B.n_slots = b->params.n_slots;
  B.pop = b->pop;
  B.rows = b->params.ga.rows;
  B.cols = b->params.ga.cols;
  B.islands = b->params.ga.islands;
  B.mig_k = b->params.ga.mig_k;
  B.mig_interval = b->params.ga.mig_interval;
  B.pc = b->params.ga.pc;
  B.pm = b->params.ga.pm;
  return B;
}

template <int MAXM>
int batch_generation_launches(const ffs_batch *b, const BatchArgs &B, hipStream_t s, bool timed) {
  const ffs_batch_params &p = b->params;
  const int K = p.ga.rows * p.ga.cols;
  const int isl_total = p.n_slots * p.ga.islands;
  const int n_cls = batch_classes(&p);
  hipError_t e = hipSuccess;
  // one launch per profile size class, each with that class's LDS
  for (int c = 0; c < n_cls && e == hipSuccess; ++c) {
    const size_t shmem = lds_bytes(p.max_genes, b->lds_slots >> (n_cls - 1 - c));
    if (p.schedule == FFS_SCHEDULE_ISLAND)
      e = launch(timed ? 4 : -1, batch_generation_kernel<MAXM, true>, dim3(b->blocks), dim3(kWave),
                 shmem, s, B, c);
    else
      e = launch(timed ? 4 : -1, batch_generation_kernel<MAXM, false>, dim3(b->blocks),
                 dim3(kWave), shmem, s, B, c);
  }
  if (e == hipSuccess && p.schedule != FFS_SCHEDULE_ISLAND)
    e = launch(-1, batch_replace_kernel, dim3(isl_total), dim3(256), 0, s, B);
  if (e == hipSuccess && p.ga.mig_interval > 0 && p.ga.mig_k > 0 && p.ga.islands > 1) {
    e = launch(-1, batch_migrate_collect_kernel, dim3(isl_total), dim3(256), (size_t)K, s, B);
    if (e == hipSuccess)
      e = launch(-1, batch_migrate_apply_kernel, dim3(isl_total), dim3(256), (size_t)K, s, B);
  }
  if (e == hipSuccess)
    e = launch(-1, batch_advance_kernel, dim3((p.n_slots + 255) / 256), dim3(256), 0, s, B);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

int batch_generation_any(const ffs_batch *b, const BatchArgs &B, hipStream_t s, bool timed) {
  switch (b->omp) {
    case 4: return batch_generation_launches<4>(b, B, s, timed);
    case 8: return batch_generation_launches<8>(b, B, s, timed);
    default: return batch_generation_launches<16>(b, B, s, timed);
  }
}

template <int MAXM>
void set_batch_lds_limits() {
  static bool done = false;
  if (done) return;
  done = true;
  const int lim = max_lds_bytes();
  (void)hipFuncSetAttribute((const void *)batch_generation_kernel<MAXM, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)batch_generation_kernel<MAXM, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void *)batch_init_kernel<MAXM>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

template <int MAXM>
int batch_init_launch(const ffs_batch *b, const BatchArgs &B, int slot, const BatchLayout &L,
                      hipStream_t s) {
  set_batch_lds_limits<MAXM>();
  const ffs_batch_params &p = b->params;
  const size_t shmem = lds_bytes(p.max_genes, b->lds_slots);
  const int grid = b->pop < b->blocks ? b->pop : b->blocks;
  if (launch(-1, batch_init_kernel<MAXM>, dim3(grid), dim3(kWave), shmem, s, B, slot) != hipSuccess ||
      launch(-1, batch_class_kernel, dim3(1), dim3(kWave), 0, s, B, slot, batch_classes(&p),
             b->lds_slots) != hipSuccess)
    return FFS_E_DEVICE;
  uint8_t *base = L.slot_base + L.slot_stride * slot;
  const int n = b->n_genes[slot];
  if (launch(-1, elite_init_kernel, dim3(p.ga.islands), dim3(256), 0, s,
             (const int32_t *)(base + L.off_prio[0]), (const int64_t *)(base + L.off_obj[0]),
             (int32_t *)(base + L.off_elite), (int64_t *)(base + L.off_eobj),
             p.ga.rows * p.ga.cols, n) != hipSuccess)
    return FFS_E_DEVICE;
  return FFS_OK;
}

// Body of ffs_decode and ffs_decode_noalloc: checks, header cleared (by a
// memset, or by a kernel for callers that may capture the call in a graph),
// instance packed, population decoded.
int decode_job_vectors(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
                       int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
                       void *workspace, size_t workspace_bytes, hipStream_t s,
                       bool clear_by_kernel) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (inst->horizon < 1 || pop < 0 || (pop > 0 && (!obj || (!prio && inst->n_active > 0))) ||
      ((start == nullptr) != (mach == nullptr)))
    return FFS_E_INVAL;
  if (pop == 0) return FFS_OK;
  const int cap = resolve_cap(inst, lds_slots);
  if (lds_bytes(inst->n_active, cap) > (size_t)max_lds_bytes())
    return FFS_E_UNSUPPORTED;
  if (!workspace || workspace_bytes < decode_layout(nullptr, inst, pop, cap).total)
    return FFS_E_WORKSPACE;
  DecodeLayout L = decode_layout(workspace, inst, pop, cap);
  if (clear_by_kernel) {
    if (launch(-1, clear_header_kernel, dim3(1), dim3(kWave), 0, s, L.hdr) != hipSuccess)
      return FFS_E_DEVICE;
  } else if ((rc = clear_header(L.hdr, s))) {
    return rc;
  }
  if ((rc = pack(inst, L.pq, s))) return rc;
  switch (omp_of(inst->o_max)) {
    case 4:
      set_lds_limits<4>();
      return run_decode<4>(inst, prio, pop, obj, start, mach, work, cap, L, s);
    case 8:
      set_lds_limits<8>();
      return run_decode<8>(inst, prio, pop, obj, start, mach, work, cap, L, s);
    default:
      set_lds_limits<16>();
      return run_decode<16>(inst, prio, pop, obj, start, mach, work, cap, L, s);
  }
}

// Address of this GPU's copy of the no-allocation decode's scratch buffer,
// looked up once per device (each GPU holds the array at its own address; the
// array's name in host code is only a stand-in for the symbol).
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FFS_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FFS_E_DEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FFS_OK;
}

// Body of reschedule and reschedule_static.
int reschedule_any(const ffs_instance *prev, const int32_t *plan_start, const int32_t *plan_mach,
                   int32_t rs, int32_t n_new, const int32_t *new_proc, const int32_t *new_power,
                   const int32_t *new_release, const int32_t *new_due, ffs_instance *next,
                   void *workspace, size_t workspace_bytes, hipStream_t s, bool static_mode) {
  int rc = check_host(prev);
  if (rc) return rc;
  if (!next || rs < prev->rs || n_new < 0 || (prev->n_jobs > 0 && (!plan_start || !plan_mach)) ||
      (n_new > 0 && (!new_proc || !new_power || !new_release || !new_due)) || !prev->release)
    return FFS_E_INVAL;
  if (prev->n_jobs + (int64_t)n_new >= (1 << 20) || rs >= kMaxTime) return FFS_E_UNSUPPORTED;
  if (!next->proc || !next->power || !next->release || !next->due || !next->first_stage ||
      !next->ready || !next->machine_free || !next->running || !next->active ||
      (static_mode && prev->n_jobs > 0 && !next->fixed))
    return FFS_E_INVAL;
  if (!workspace || workspace_bytes < ffs_reschedule_workspace_size(prev->n_jobs, n_new))
    return FFS_E_WORKSPACE;
  Header *h = (Header *)workspace;
  if ((rc = clear_header(h, s))) return rc;
  ReschedArgs a{prev->n_machines, prev->proc, prev->power, prev->release, prev->due,
                prev->n_jobs, prev->n_stages, prev->o_max, prev->q_max, prev->rs,
                plan_start, plan_mach, rs, n_new, new_proc, new_power, new_release, new_due,
                (int32_t *)next->proc, (int32_t *)next->power, (int32_t *)next->release,
                (int32_t *)next->due, (int32_t *)next->first_stage, (int32_t *)next->ready,
                (int32_t *)next->machine_free, (int32_t *)next->running, (int32_t *)next->active,
                prev->n_stages * prev->o_max, static_mode ? 1 : 0,
                static_mode ? (int32_t *)next->fixed : nullptr, prev->n_jobs * prev->n_stages};
  if (launch(-1, reschedule_kernel, dim3(1), dim3(1024), 0, s, a, h) != hipSuccess)
    return FFS_E_DEVICE;
  Header host;
  if ((rc = read_header(h, &host, s))) return rc;
  if ((rc = err_code(host.err))) return rc;
  if (host.horizon + (int64_t)rs >= kMaxTime) return FFS_E_UNSUPPORTED;
  next->n_jobs = prev->n_jobs + n_new;
  next->n_stages = prev->n_stages;
  next->o_max = prev->o_max;
  if (!next->n_machines) next->n_machines = prev->n_machines;
  next->q_max = prev->q_max;
  next->wt = prev->wt;
  next->rs = rs;
  next->n_running = host.n_running;
  next->n_fixed = static_mode ? host.n_fixed : 0;
  next->frozen_tardiness = host.frozen_tardiness;
  next->frozen_cmax = host.frozen_cmax;
  next->n_active = host.n_active;
  next->horizon = (int32_t)host.horizon;
  next->n_ops = host.n_ops;
  next->decode_rules = prev->decode_rules;
  return check_host(next);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

#ifndef FFS_BUILD_ID
#define FFS_BUILD_ID "unknown"
#endif
const char *ffs_build_id(void) { return FFS_BUILD_ID; }

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
             inst->o_max, inst->q_max, inst->rs, inst->n_running, inst->n_active, inst->fixed,
             inst->n_fixed};
  if (launch(-1, prepare_kernel, dim3(1), dim3(1024), 0, s, a, h) != hipSuccess) return FFS_E_DEVICE;
  Header host;
  if ((rc = read_header(h, &host, s))) return rc;
  if ((rc = err_code(host.err))) return rc;
  if (host.horizon + inst->rs >= kMaxTime) return FFS_E_UNSUPPORTED;
  inst->horizon = (int32_t)host.horizon;
  inst->n_ops = host.n_ops;
  return FFS_OK;
}

size_t ffs_decode_workspace_size(const ffs_instance *inst, int32_t pop, int32_t lds_slots) {
  if (check_host(inst) || inst->horizon < 1 || pop < 0) return 0;
  const int cap = resolve_cap(inst, lds_slots);
  return decode_layout(nullptr, inst, pop, cap).total;
}

int ffs_decode(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots, void *workspace,
               size_t workspace_bytes, void *stream) {
  return decode_job_vectors(inst, prio, pop, obj, start, mach, work, lds_slots, workspace,
                            workspace_bytes, (hipStream_t)stream, false);
}

int ffs_decode_noalloc(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
                       int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
                       void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (inst->horizon < 1 || pop < 0) return FFS_E_INVAL;
  if (pop > 0 && ffs_decode_workspace_size(inst, pop, lds_slots) > (size_t)FFS_DECODE_SCRATCH_BYTES)
    return FFS_E_WORKSPACE;
  void *ws = nullptr;
  if ((rc = static_scratch(&ws))) return rc;
  return decode_job_vectors(inst, prio, pop, obj, start, mach, work, lds_slots, ws,
                            FFS_DECODE_SCRATCH_BYTES, (hipStream_t)stream, true);
}

int ffs_decode_xy(const ffs_instance *inst, const int32_t *genes, int32_t pop, int64_t *obj,
                  int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
                  void *workspace, size_t workspace_bytes, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (inst->horizon < 1 || inst->n_ops < 0 || pop < 0 ||
      (pop > 0 && (!obj || (!genes && inst->n_ops > 0))) || ((start == nullptr) != (mach == nullptr)))
    return FFS_E_INVAL;
  if (pop == 0) return FFS_OK;
  const int cap = resolve_cap(inst, lds_slots);
  if (lds_bytes_xy(inst->n_active, inst->n_ops, inst->n_stages, inst->o_max, cap) >
      (size_t)max_lds_bytes())
    return FFS_E_UNSUPPORTED;
  if (!workspace || workspace_bytes < ffs_decode_workspace_size(inst, pop, lds_slots))
    return FFS_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  DecodeLayout L = decode_layout(workspace, inst, pop, cap);
  if ((rc = clear_header(L.hdr, s))) return rc;
  if ((rc = pack(inst, L.pq, s))) return rc;
  if ((rc = build_xy_table(inst, L.xyop, L.xyg0, s))) return rc;
  switch (omp_of(inst->o_max)) {
    case 4:
      set_lds_limits<4>();
      return run_decode_xy<4>(inst, genes, pop, obj, start, mach, work, cap, L, s);
    case 8:
      set_lds_limits<8>();
      return run_decode_xy<8>(inst, genes, pop, obj, start, mach, work, cap, L, s);
    default:
      set_lds_limits<16>();
      return run_decode_xy<16>(inst, genes, pop, obj, start, mach, work, cap, L, s);
  }
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
  return ga_layout(nullptr, inst, params, layout_cap(params, cap)).total;
}

int ga_init(ffs_ga *ga, const ffs_instance *inst, const ffs_ga_params *params, uint64_t seed,
            uint64_t shop, int32_t event, void *workspace, size_t workspace_bytes, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (!ga || inst->horizon < 1) return FFS_E_INVAL;
  if ((rc = check_ga_params(params))) return rc;
  const bool auto_cap = params->lds_slots == FFS_LDS_AUTO;
  if (auto_cap && params->encoding != 0) return FFS_E_UNSUPPORTED;
  const int cap = auto_cap ? probe_cap(inst) : resolve_cap(inst, params->lds_slots);
  const size_t lds = params->encoding == 1
                         ? lds_bytes_xy(inst->n_active, inst->n_ops, inst->n_stages, inst->o_max, cap)
                         : lds_bytes(inst->n_active, cap);
  if (lds > (size_t)max_lds_bytes()) return FFS_E_UNSUPPORTED;
  const size_t need = ffs_ga_workspace_size(inst, params);
  if (!workspace || workspace_bytes < need) return FFS_E_WORKSPACE;
  memset(ga, 0, sizeof(*ga));
  ga->params = *params;
  ga->n_genes = (int32_t)chrom_len(inst, params);
  ga->pop = params->islands * params->rows * params->cols;
  ga->seed = seed;
  ga->shop = shop;
  ga->event = event;
  ga->generation = 0;
  ga->cur = 0;
  ga->island_groups = 0;
  ga->narrow_lds = 0;
  ga->workspace = workspace;
  ga->workspace_bytes = workspace_bytes;
  ga->lds_slots = cap;
  ga->n_jobs = inst->n_jobs;
  ga->horizon = inst->horizon;
  hipStream_t s = (hipStream_t)stream;
  GaLayout L = ga_layout(workspace, inst, params, layout_cap(params, cap));
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
  switch (omp_of(inst->o_max)) {
    case 4:
      set_lds_limits<4>();
      return ga_init_impl<4>(ga, inst, L, s, auto_cap);
    case 8:
      set_lds_limits<8>();
      return ga_init_impl<8>(ga, inst, L, s, auto_cap);
    default:
      set_lds_limits<16>();
      return ga_init_impl<16>(ga, inst, L, s, auto_cap);
  }
}

int ga_step(ffs_ga *ga, const ffs_instance *inst, int32_t n_generations, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (!ga || !ga->workspace || n_generations < 0 || chrom_len(inst, &ga->params) != ga->n_genes ||
      inst->n_jobs != ga->n_jobs || inst->horizon != ga->horizon)
    return FFS_E_INVAL;
  if (inst->n_active == 0) {
    ga->generation += n_generations;
    return FFS_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const int span = span_begin(s);
  switch (omp_of(inst->o_max)) {
    case 4: rc = ga_step_impl<4>(ga, inst, n_generations, s); break;
    case 8: rc = ga_step_impl<8>(ga, inst, n_generations, s); break;
    default: rc = ga_step_impl<16>(ga, inst, n_generations, s);
  }
  span_end(span, s, rc == FFS_OK ? n_generations : 0);
  return rc;
}

int ga_set_island_groups(int32_t groups) {
  if (groups < 0 || groups > kMaxGroups) return FFS_E_INVAL;
  g_island_groups.store(groups);
  if (groups == 1) return FFS_OK;
  std::lock_guard<std::mutex> lk(g_group_mu);
  GroupStreams *GS = nullptr;
  return group_streams(&GS);
}

int sg_score(const ffs_surrogate *model, const float *table, int32_t n_genes, const int32_t *prio,
             int32_t count, float *y, void *stream) {
  if (!model || !model->theta || !table || !prio || !y || n_genes < 1 ||
      n_genes > FFS_SG_MAX_GENES || count < 0)
    return FFS_E_INVAL;
  if (launch(-1, sg_score_kernel, dim3(count), dim3(kWave), 0, (hipStream_t)stream, table,
             (const float *)model->theta, n_genes, prio, y) != hipSuccess)
    return FFS_E_DEVICE;
  return FFS_OK;
}

int ga_step_screened(ffs_ga *ga, const ffs_instance *inst, const ffs_surrogate *model,
                     const float *table, int32_t variants, int32_t n_generations, float *scores,
                     int32_t *choice, void *stream) {
  int rc = check_host(inst);
  if (rc) return rc;
  if (ga && (ga->params.encoding != 0 || ga->params.scheme != FFS_GA_HYBRID))
    return FFS_E_UNSUPPORTED;
  if (!ga || !ga->workspace || n_generations < 0 || inst->n_active != ga->n_genes ||
      inst->n_jobs != ga->n_jobs || inst->horizon != ga->horizon || !model || !model->theta ||
      !table || variants < 1 || variants > FFS_SG_MAX_VARIANTS ||
      inst->n_active > FFS_SG_MAX_GENES)
    return FFS_E_INVAL;
  if (inst->n_active == 0) {
    ga->generation += n_generations;
    return FFS_OK;
  }
  const Screen scr{table, model->theta, variants, scores, choice};
  hipStream_t s = (hipStream_t)stream;
  switch (omp_of(inst->o_max)) {
    case 4: return ga_step_impl<4>(ga, inst, n_generations, s, &scr);
    case 8: return ga_step_impl<8>(ga, inst, n_generations, s, &scr);
    default: return ga_step_impl<16>(ga, inst, n_generations, s, &scr);
  }
}

int ga_view(const ffs_ga *ga, ffs_ga_view *view) {
  if (!ga || !view || !ga->workspace) return FFS_E_INVAL;
  view->prio = ga->prio[ga->cur];
  view->obj = ga->obj[ga->cur];
  view->elite = ga->elite;
  view->elite_obj = ga->elite_obj;
  view->work = (int64_t *)&((Header *)ga->workspace)->work;
  view->e_max = &((Header *)ga->workspace)->e_max;
  view->overflows = (int64_t *)&((Header *)ga->workspace)->overflows;
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
  return reschedule_any(prev, plan_start, plan_mach, rs, n_new, new_proc, new_power, new_release,
                        new_due, next, workspace, workspace_bytes, (hipStream_t)stream, false);
}

int reschedule_static(const ffs_instance *prev, const int32_t *plan_start,
                      const int32_t *plan_mach, int32_t rs, int32_t n_new,
                      const int32_t *new_proc, const int32_t *new_power,
                      const int32_t *new_release, const int32_t *new_due, ffs_instance *next,
                      void *workspace, size_t workspace_bytes, void *stream) {
  return reschedule_any(prev, plan_start, plan_mach, rs, n_new, new_proc, new_power, new_release,
                        new_due, next, workspace, workspace_bytes, (hipStream_t)stream, true);
}

size_t ffs_batch_workspace_size(const ffs_batch_params *params) {
  if (check_batch_params(params)) return 0;
  return batch_layout(nullptr, params).total;
}

int ga_batch_create(ffs_batch *b, const ffs_batch_params *params, void *workspace,
                    size_t workspace_bytes, void *stream) {
  if (!b) return FFS_E_INVAL;
  int rc = check_batch_params(params);
  if (rc) return rc;
  const size_t need = ffs_batch_workspace_size(params);
  if (!workspace || workspace_bytes < need) return FFS_E_WORKSPACE;
  memset(b, 0, sizeof(*b));
  b->params = *params;
  b->pop = params->ga.islands * params->ga.rows * params->ga.cols;
  b->lds_slots = batch_cap(params);
  b->blocks = batch_blocks(params);
  b->omp = omp_of(params->o_max);
  b->workspace = workspace;
  b->workspace_bytes = workspace_bytes;
  if (lds_bytes(params->max_genes, b->lds_slots) > (size_t)max_lds_bytes())
    return FFS_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  BatchLayout L = batch_layout(workspace, params);
  if ((rc = clear_header(L.hdr, s))) return rc;
  std::vector<BatchSlot> slots((size_t)params->n_slots);
  memset(slots.data(), 0, sizeof(BatchSlot) * slots.size());
  if (hipMemcpyAsync(L.slots, slots.data(), sizeof(BatchSlot) * slots.size(),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFS_E_DEVICE;
  return FFS_OK;
}

int ga_batch_set(ffs_batch *b, int32_t slot, const ffs_instance *inst, uint64_t seed,
                 uint64_t shop, int32_t event, void *stream) {
  if (!b || !b->workspace || slot < 0 || slot >= b->params.n_slots) return FFS_E_INVAL;
  int rc = check_host(inst);
  if (rc) return rc;
  if (inst->horizon < 1) return FFS_E_INVAL;
  const ffs_batch_params &p = b->params;
  if (inst->n_jobs > p.max_jobs || inst->n_active > p.max_genes || inst->n_stages > p.max_stages ||
      omp_of(inst->o_max) > b->omp || inst->horizon > p.max_horizon)
    return FFS_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  BatchLayout L = batch_layout(b->workspace, &p);
  uint8_t *base = L.slot_base + L.slot_stride * slot;
  // pack the instance's rows at the batch's row width
  if ((rc = pack(inst, (uint32_t *)(base + L.off_pq), s, b->omp))) return rc;
  BatchSlot S;
  memset(&S, 0, sizeof(S));
  S.I = make_dinst(inst, (const uint32_t *)(base + L.off_pq), b->omp);
  for (int k = 0; k < 2; ++k) {
    S.prio[k] = (int32_t *)(base + L.off_prio[k]);
    S.obj[k] = (int64_t *)(base + L.off_obj[k]);
  }
  S.elite = (int32_t *)(base + L.off_elite);
  S.elite_obj = (int64_t *)(base + L.off_eobj);
  S.stage_prio = (int32_t *)(base + L.off_sprio);
  S.stage_obj = (int64_t *)(base + L.off_sobj);
  S.seed = seed;
  S.shop = shop;
  S.event = event;
  S.gen = 0;
  S.active = 1;
  const int h = (int)align_up((size_t)inst->horizon, 64);
  S.cap = b->lds_slots < h ? b->lds_slots : h;
  if (hipMemcpyAsync(L.slots + slot, &S, sizeof(S), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFS_E_DEVICE;
  b->active[slot] = 1;
  b->generation[slot] = 0;
  b->n_genes[slot] = inst->n_active;
  if (inst->n_active == 0) {
    std::vector<int64_t> o((size_t)b->pop, (int64_t)inst->wt * inst->frozen_tardiness + inst->frozen_cmax);
    if (hipMemcpyAsync(S.obj[0], o.data(), o.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(S.elite_obj, o.data(), (size_t)p.ga.islands * 8, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FFS_E_DEVICE;
    return FFS_OK;
  }
  const BatchArgs B = batch_args(b, L);
  switch (b->omp) {
    case 4: return batch_init_launch<4>(b, B, slot, L, s);
    case 8: return batch_init_launch<8>(b, B, slot, L, s);
    default: return batch_init_launch<16>(b, B, slot, L, s);
  }
}

int ga_batch_clear(ffs_batch *b, int32_t slot, void *stream) {
  if (!b || !b->workspace || slot < 0 || slot >= b->params.n_slots) return FFS_E_INVAL;
  BatchLayout L = batch_layout(b->workspace, &b->params);
  const int32_t zero = 0;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&L.slots[slot].active, &zero, sizeof(zero), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFS_E_DEVICE;
  b->active[slot] = 0;
  return FFS_OK;
}

int ga_batch_step(ffs_batch *b, int32_t n_generations, void *stream) {
  if (!b || !b->workspace || n_generations < 0) return FFS_E_INVAL;
  hipStream_t s = (hipStream_t)stream;
  BatchLayout L = batch_layout(b->workspace, &b->params);
  const BatchArgs B = batch_args(b, L);
  switch (b->omp) {
    case 4: set_batch_lds_limits<4>(); break;
    case 8: set_batch_lds_limits<8>(); break;
    default: set_batch_lds_limits<16>(); break;
  }
  if (b->params.use_graph) {
    if (!s) return FFS_E_INVAL;  // the legacy default stream cannot be captured
    if (!b->graph_exec) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ge = nullptr;
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return FFS_E_DEVICE;
      const int rc = batch_generation_any(b, B, s, false);
      if (hipStreamEndCapture(s, &g) != hipSuccess || rc) return rc ? rc : FFS_E_DEVICE;
      if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return FFS_E_DEVICE;
      }
      b->graph = g;
      b->graph_exec = ge;
      b->graph_stream = s;
    }
    for (int32_t k = 0; k < n_generations; ++k)
      if (hipGraphLaunch((hipGraphExec_t)b->graph_exec, s) != hipSuccess) return FFS_E_DEVICE;
  } else {
    for (int32_t k = 0; k < n_generations; ++k) {
      const int rc = batch_generation_any(b, B, s, true);
      if (rc) return rc;
    }
  }
  for (int d = 0; d < b->params.n_slots; ++d)
    if (b->active[d]) b->generation[d] += n_generations;
  return FFS_OK;
}

int ga_batch_best(const ffs_batch *b, int32_t slot, int32_t *prio_out, int64_t *obj_out,
                  void *stream) {
  if (!b || !b->workspace || slot < 0 || slot >= b->params.n_slots || !b->active[slot] || !obj_out)
    return FFS_E_INVAL;
  BatchLayout L = batch_layout(b->workspace, &b->params);
  uint8_t *base = L.slot_base + L.slot_stride * slot;
  hipError_t e = launch(-1, best_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream,
                        (const int32_t *)(base + L.off_elite), (const int64_t *)(base + L.off_eobj),
                        b->params.ga.islands, b->n_genes[slot], prio_out, obj_out);
  return e == hipSuccess ? FFS_OK : FFS_E_DEVICE;
}

int ga_batch_view(const ffs_batch *b, int32_t slot, ffs_ga_view *view) {
  if (!b || !b->workspace || slot < 0 || slot >= b->params.n_slots || !view) return FFS_E_INVAL;
  BatchLayout L = batch_layout(b->workspace, &b->params);
  uint8_t *base = L.slot_base + L.slot_stride * slot;
  const int cur = b->generation[slot] & 1;
  view->prio = (int32_t *)(base + L.off_prio[cur]);
  view->obj = (int64_t *)(base + L.off_obj[cur]);
  view->elite = (int32_t *)(base + L.off_elite);
  view->elite_obj = (int64_t *)(base + L.off_eobj);
  view->work = (int64_t *)&L.hdr->work;
  return FFS_OK;
}

int ga_batch_destroy(ffs_batch *b) {
  if (!b) return FFS_E_INVAL;
  if (b->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)b->graph_exec);
  if (b->graph) (void)hipGraphDestroy((hipGraph_t)b->graph);
  b->graph_exec = nullptr;
  b->graph = nullptr;
  return FFS_OK;
}

int ffs_timing_enable(int32_t families) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (families) {
    for (int f = 0; f < kTimingFamilies; ++f) {
      if (g_timing.ev[f].empty()) {
        g_timing.ev[f].resize(2 * kTimingPairs);
        for (auto &e : g_timing.ev[f])
          if (hipEventCreate(&e) != hipSuccess) return FFS_E_DEVICE;
      }
      g_timing.used[f] = 0;
      g_timing.ms[f] = 0;
      g_timing.launches[f] = 0;
      g_timing.seen[f] = 0;
    }
  }
  g_timing.on = families != 0;
  g_timing.mask = (uint32_t)families;
  return FFS_OK;
}

int ffs_timing_every(int32_t every) {
  if (every < 1) return FFS_E_INVAL;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  g_timing.every = every;
  return FFS_OK;
}

int ffs_timing_read(int32_t family, double *total_ms, int64_t *launches) {
  if (family < 0 || family >= kTimingFamilies || !total_ms || !launches) return FFS_E_INVAL;
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
