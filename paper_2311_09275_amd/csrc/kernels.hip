// kernels.hip -- gfx950 kernels of the many-replica Metropolis annealer.
//
// Method (one replica): visit colour classes 0..C-1; for each vertex i of
// the class compute k = s_i h_i (flipping s_i changes E by 2k); accept when
// k <= 0, otherwise when the u32 draw is below Tq(beta_t, k); on a flip add
// -2 w_ij s_i(new) to every neighbour's field.  The classes come from a
// proper colouring, so all vertices of one class are updated in parallel
// without races on their own state; pushes into neighbour fields are
// integer atomics and therefore order independent.  The best cut is taken
// over end-of-sweep states (strict improvement).
//
// Random numbers: word j of Philox4x32-10 with key = seed and counter =
// (t, g, r, tag) serves the j-th vertex of group g -- four consecutive
// same-colour vertices, groups numbered in class order.  One block call therefore feeds four attempts of one
// replica, which lets a single replica be a unit of parallel work.
//
// Three kernel families compute identical results:
//   plain  state in HBM, [position][replica] so a wave's 64 lanes touch 64
//          consecutive replicas; one launch per colour pass.
//   field  persistent: a workgroup owns G replicas of one problem for all
//          sweeps, the packed word (h << 1) | spin_bit of every vertex lives
//          in LDS; only workgroup barriers separate colour passes.
//   msc    persistent multispin: bit b of a 32-bit word is the spin of
//          replica 32w+b; unsatisfied bonds of 32 replicas are counted with
//          bit-sliced adders, no field array; +-1 weights only.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_types.h"
#include "kernels.h"

namespace ising {
namespace {

// ---------------------------------------------------------------- Philox
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
// products; key advanced by the Weyl constants between rounds.  From the
// fourth round on every word differs per lane, and each new word's two
// XORs are one three-input bitwise operation (truth table 0x96); the first
// three rounds keep plain XORs, which the compiler folds where words are
// the same for the whole wave.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                          uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
    const uint32_t n0 = i < 3 ? (uint32_t)(p1 >> 32) ^ c1 ^ k0 : xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = i < 3 ? (uint32_t)(p0 >> 32) ^ c3 ^ k1 : xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return make_uint4(c0, c1, c2, c3);
}

// Eight 32x32->64 products p[2b] = m0 a[2b], p[2b+1] = m1 a[2b+1], issued
// back to back: one statement, so that the eight independent chains of four
// Philox blocks stay interleaved (the instruction scheduler would otherwise
// order the blocks one after another, leaving a single wave waiting on
// each product).  The carry-out SGPR pair of the instruction is unused.
__device__ __forceinline__ void mul8_u64(uint64_t (&p)[8], const uint32_t (&a)[8], uint32_t m0,
                                         uint32_t m1) {
  uint64_t carry;
  asm("v_mad_u64_u32 %0, %8, %9, %17, 0\n\t"
      "v_mad_u64_u32 %1, %8, %10, %18, 0\n\t"
      "v_mad_u64_u32 %2, %8, %11, %17, 0\n\t"
      "v_mad_u64_u32 %3, %8, %12, %18, 0\n\t"
      "v_mad_u64_u32 %4, %8, %13, %17, 0\n\t"
      "v_mad_u64_u32 %5, %8, %14, %18, 0\n\t"
      "v_mad_u64_u32 %6, %8, %15, %17, 0\n\t"
      "v_mad_u64_u32 %7, %8, %16, %18, 0"
      : "=&v"(p[0]), "=&v"(p[1]), "=&v"(p[2]), "=&v"(p[3]), "=&v"(p[4]), "=&v"(p[5]),
        "=&v"(p[6]), "=&v"(p[7]), "=&s"(carry)
      : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7]),
        "s"(kPhiloxM0), "s"(kPhiloxM1));
}

// Four blocks of counters (c0, c1, c2[b], c3) under one key, computed round
// by round across the blocks.  The first three rounds are left to the
// compiler, which folds the products of words that are the same for the
// whole wave; from the fourth round on every word differs per lane.
__device__ __forceinline__ void philox10_x4(uint32_t c0, uint32_t c1, const uint32_t (&c2)[4],
                                            uint32_t c3, uint32_t k0, uint32_t k1,
                                            uint4 (&out)[4]) {
  uint32_t a0[4], a1[4], a2[4], a3[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    a0[b] = c0;
    a1[b] = c1;
    a2[b] = c2[b];
    a3[b] = c3;
  }
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    uint64_t p[8];
    if (i < 3) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        p[2 * b] = (uint64_t)kPhiloxM0 * a0[b];
        p[2 * b + 1] = (uint64_t)kPhiloxM1 * a2[b];
      }
    } else {
      const uint32_t in[8] = {a0[0], a2[0], a0[1], a2[1], a0[2], a2[2], a0[3], a2[3]};
      mul8_u64(p, in, kPhiloxM0, kPhiloxM1);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint64_t p0 = p[2 * b], p1 = p[2 * b + 1];
      const uint32_t n0 = i < 3 ? (uint32_t)(p1 >> 32) ^ a1[b] ^ k0 : xor3((uint32_t)(p1 >> 32), a1[b], k0);
      const uint32_t n2 = i < 3 ? (uint32_t)(p0 >> 32) ^ a3[b] ^ k1 : xor3((uint32_t)(p0 >> 32), a3[b], k1);
      a1[b] = (uint32_t)p1;
      a3[b] = (uint32_t)p0;
      a0[b] = n0;
      a2[b] = n2;
    }
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) out[b] = make_uint4(a0[b], a1[b], a2[b], a3[b]);
}

// The block of a four-vertex group: counter (sweep, group ordinal,
// replica, tag), key (seed low, seed high); the group's j-th vertex uses
// word j.  The ordinal counts runs of four same-colour vertices in class
// order, which is the group's index in the position layout.  Sweep,
// replica and tag are the same for a whole wave, so with the group in word
// 1 the first round's products and one product of each of the next two
// rounds do not depend on the lane.
__device__ __forceinline__ uint4 group_block(uint32_t group, uint32_t t, uint32_t r,
                                             uint32_t tag, uint32_t k0, uint32_t k1) {
  return philox10(t, group, r, tag, k0, k1);
}

// Pointers fetched from a descriptor are generic; re-qualifying them as
// global lets the compiler emit global (not flat) memory instructions.
#define GLOBAL_AS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GLOBAL_AS T* gconst(const T* p) {
  return (const GLOBAL_AS T*)p;
}
template <class T>
__device__ __forceinline__ GLOBAL_AS T* gmut(T* p) {
  return (GLOBAL_AS T*)p;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pick(const uint4& x, int j) {
  return j == 0 ? x.x : j == 1 ? x.y : j == 2 ? x.z : x.w;
}

// ---------------------------------------------------------------- waves
// Sum over the wave, returned in every lane.  DPP steps reduce each row of
// 16 lanes (quad swaps, half-row and row mirrors) without an LDS round
// trip; the four row sums are then read out as scalars.
__device__ __forceinline__ int wave_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Accept test for k > 0 against a threshold row holding Tq-1 for
// k = 1..len (len = kAcceptAll when beta = 0).
__device__ __forceinline__ bool accept_pos(int k, int len, uint32_t draw,
                                           const uint32_t* row) {
  return len < 0 || (k <= len && draw <= row[k - 1]);
}

// Encode four +-1 spins (bit set = +1) as four int8 bytes.
__device__ __forceinline__ uint32_t spins_to_bytes(uint32_t bits4) {
  uint32_t out = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) out |= ((bits4 >> j) & 1u ? 0x01u : 0xFFu) << (8 * j);
  return out;
}

// ================================================================ plain
// Grid: one lane per (group, replica), replica fastest.

__global__ void k_plain_init(PlainDev P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_grp = P.n_pad >> 2;
  if (idx >= (int64_t)n_grp * P.R) return;
  const int g = (int)(idx / P.R), r = (int)(idx - (int64_t)g * P.R);
  const int gw = P.grp[g];
  const int cnt = (gw >> kGroupCountShift) + 1;
  uint32_t bits = 0;
  if (P.init_spins) {
    for (int j = 0; j < cnt; ++j)
      bits |= (P.init_spins[(int64_t)r * P.n_pad + 4 * g + j] > 0 ? 1u : 0u) << j;
  } else {
    const uint4 x = group_block((uint32_t)g, 0, r, kTagInit, P.seed_lo, P.seed_hi);
    bits = (x.x >> 31) | ((x.y >> 31) << 1) | ((x.z >> 31) << 2) | ((x.w >> 31) << 3);
  }
  for (int j = 0; j < 4; ++j)
    P.spins[(int64_t)(4 * g + j) * P.R + r] = (j >= cnt || ((bits >> j) & 1u)) ? 1 : -1;
}

// h_p = -sum_q w_pq s_q, and the energy sum -1/2 sum_p s_p h_p per replica.
__global__ void k_plain_fields(PlainDev P) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)P.n_pad * P.R) return;
  const int p = (int)(idx / P.R), r = (int)(idx - (int64_t)p * P.R);
  // with local fields h_p = -sum w s + 2 b_p, and the energy sum takes
  // s (h + 2 b): E = sum w s s - 2 sum b s = -1/2 sum s (h + 2 b)
  const int bf = P.bfield ? 2 * P.bfield[p] : 0;
  int h = bf;
  for (int a = P.row[p]; a < P.row[p + 1]; ++a)
    h -= P.wgt[a] * (int)P.spins[(int64_t)P.adj[a] * P.R + r];
  P.field[idx] = h;
  const int sh = (int)P.spins[idx] * (h + bf);
  if (sh != 0) atomicAdd(&P.eacc[r], sh);
}

__global__ void k_plain_init_best(PlainDev P) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P.R) return;
  const int E = -P.eacc[r] / 2;
  P.eacc[r] = 0;
  P.energy[r] = E;
  P.best_cut[r] = (P.W - E) / 2;
  P.best_sweep[r] = -1;
  P.snap[r] = -1;
  P.accepts[r] = 0;
}

// One colour pass of sweep t over the groups [g0, g1).
__global__ void k_plain_sweep(PlainDev P, int t, int g0, int g1) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(g1 - g0) * P.R) return;
  const int gl = (int)(idx / P.R), r = (int)(idx - (int64_t)gl * P.R);
  const int g = g0 + gl;
  const int gw = P.grp[g];
  const int cnt = (gw >> kGroupCountShift) + 1;
  const int ri = P.temp ? P.temp[r] : t;  // parallel tempering: its temperature's row
  const int len = P.tq_len[ri];
  const uint32_t* row = P.tq + P.tq_off[ri];
  const bool snap = P.snap[r] == t - 1;
  int s[4], k[4];
  bool need = false;
  for (int j = 0; j < 4; ++j) {
    if (j < cnt) {
      const int64_t o = (int64_t)(4 * g + j) * P.R + r;
      s[j] = P.spins[o];
      k[j] = s[j] * P.field[o];
      if (snap) P.best[o] = (int8_t)s[j];
      need |= k[j] > 0 && k[j] <= len;
    }
  }
  uint4 x = make_uint4(0, 0, 0, 0);
  if (need) x = group_block((uint32_t)g, t, r, kTagSweep, P.seed_lo, P.seed_hi);
  int dE = 0, nacc = 0;
  for (int j = 0; j < cnt; ++j) {
    if (k[j] <= 0 || accept_pos(k[j], len, pick(x, j), row)) {
      const int p = 4 * g + j;
      const int sn = -s[j];
      P.spins[(int64_t)p * P.R + r] = (int8_t)sn;
      dE += 2 * k[j];
      ++nacc;
      for (int a = P.row[p]; a < P.row[p + 1]; ++a)
        atomicAdd(&P.field[(int64_t)P.adj[a] * P.R + r], -2 * P.wgt[a] * sn);
    }
  }
  if (dE != 0) atomicAdd(&P.eacc[r], dE);
  if (nacc != 0) atomicAdd(&P.accepts[r], (unsigned long long)nacc);
}

// End of sweep t: energy, cut, strict best update.
__global__ void k_plain_eos(PlainDev P, int t, int S) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P.R) return;
  const int E = P.energy[r] + P.eacc[r];
  P.eacc[r] = 0;
  P.energy[r] = E;
  const int cut = (P.W - E) / 2;
  if (cut > P.best_cut[r]) {
    P.best_cut[r] = cut;
    P.best_sweep[r] = t;
    P.snap[r] = t;
  }
  if (P.flags & kJobTrace) P.trace[(int64_t)t * P.R + r] = E;
  (void)S;
}

// The last sweep improved: its end state is the best state.
__global__ void k_plain_flush(PlainDev P, int last) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)P.n_pad * P.R) return;
  const int r = (int)(idx % P.R);
  if (P.snap[r] == last) P.best[idx] = P.spins[idx];
}

// ================================================================ field
// Persistent kernel: workgroups pull (job, replica block) units from eight
// lists (one per XCD, by blockIdx % 8) and steal from the others once their
// own is empty.  Unit processing is entirely workgroup-local.
//
// LDS of a unit: the state words of its G replicas, two threshold rows
// (current and next sweep), and the group descriptors: group word (first
// vertex and slot count), adjacency base and four 8-bit slot degrees.

struct FieldShared {
  int32_t unit;
  int32_t eacc[4][kMaxReplicasPerBlock];  // [sweep % 3] energy change; [3] init
  int32_t nacc[kMaxReplicasPerBlock];
};

struct UnitLds {
  uint32_t* tq;     // FIELD: [row_chunk][row words] rows; MSC: [2][kw] (t even, odd)
  int32_t* cls;     // [2C] first and end group of each class (FIELD)
  int32_t* gword;   // [n_grp]
  int32_t* gbase;   // [n_grp]
  uint32_t* gdeg;   // [n_grp]
  uint16_t* adj16;  // staged adjacency.  CSR form: [2m] entries
                    // (position << 1) | (w > 0).  Degree-4 form: [n_grp]
                    // 48-byte group blocks (kDeg4BlockWords)
  uint32_t* flips;  // [BLOCK/64][256] per-wave lists of flipped vertices (CSR form)
};

// Staged adjacency forms (the kernel's ADJ parameter).
constexpr int kAdjHbm = 0;      // {position, w} pairs read from HBM
constexpr int kAdjLds = 1;      // 16-bit CSR entries in LDS, wave-compacted pushes
constexpr int kAdjLdsDeg4 = 2;  // every vertex of degree 4: 32 bytes per group
constexpr int kAdjPerJob = 3;   // each job's own form (JobDev::adj_form), for mixed batches
constexpr int kAdjHbmDeg4 = 4;  // the degree-4 blocks read from HBM (graphs too large for LDS)

__device__ __forceinline__ UnitLds unit_lds(uint32_t* smem, int words, int tq_words,
                                            int cls_words, int n_grp) {
  UnitLds u;
  u.tq = smem + words;
  u.cls = reinterpret_cast<int32_t*>(u.tq + tq_words);
  u.gword = u.cls + cls_words;
  u.gbase = u.gword + n_grp;
  u.gdeg = reinterpret_cast<uint32_t*>(u.gbase + n_grp);
  // 16-byte aligned so that a group's sixteen degree-4 entries are two
  // 128-bit reads (and four general entries one 64-bit read)
  const int used = words + tq_words + cls_words + 3 * n_grp;
  u.adj16 = reinterpret_cast<uint16_t*>(u.gdeg + n_grp + ((4 - (used & 3)) & 3));
  u.flips = nullptr;
  return u;
}

// Flip lists follow the staged adjacency (m entries of 2 x 16 bits).
__device__ __forceinline__ void place_flip_lists(UnitLds& u, int m) {
  u.flips = reinterpret_cast<uint32_t*>(u.adj16) + m + 1;
}

// Compact adjacency of a unit-weight graph with fewer than 2^15 positions.
// Global -> LDS copy of n elements, dst[i] = f(src[i]), with eight loads of
// every thread in flight at a time: a plain strided loop waits for each
// load before it issues the next, and a unit's staging would then cost one
// memory latency per element per thread.
template <class T, class D, class F>
__device__ __forceinline__ void copy_in(D* dst, const T* src, int n, F f) {
  const GLOBAL_AS T* s = gconst(src);
  const int nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < n; i0 += 8 * nt) {
    // indices past the end re-read the last element (every load is
    // unconditional, so the values stay in registers)
    T v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = s[min(i0 + k * nt, n - 1)];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + k * nt < n) dst[i0 + k * nt] = f(v[k]);
  }
}
template <class T>
__device__ __forceinline__ void copy_in(T* dst, const T* src, int n) {
  copy_in(dst, src, n, [](const T& x) { return x; });
}

__device__ __forceinline__ void stage_adjacency(const JobDev& J, const UnitLds& u) {
  copy_in(u.adj16, J.adjm, 2 * J.M, [](uint32_t x) { return (uint16_t)x; });
}

// Degree-4 form: the unit's copy of the 48-byte group blocks
// (kDeg4BlockWords), built on the host.
__device__ __forceinline__ void stage_adjacency_deg4(const JobDev& J, UnitLds& u) {
  copy_in(reinterpret_cast<u32x4*>(u.adj16), reinterpret_cast<const u32x4*>(J.adj4),
          3 * (J.n_pad >> 2));
}

__device__ __forceinline__ void stage_row(const JobDev& J, int t, uint32_t* buf) {
  if (t >= J.t_end) return;
  const int len = gconst(J.tq_len)[t];
  const GLOBAL_AS uint32_t* src = gconst(J.tq) + gconst(J.tq_off)[t];
  for (int i = threadIdx.x; i < len; i += blockDim.x) buf[(t & 1) * J.kw + i] = src[i];
}

// FIELD rows (rw words each, see JobDev::tqp and JobDev::tqb) of sweeps
// t .. t+n-1, one contiguous copy.
__device__ __forceinline__ void stage_row_chunk(const uint32_t* rows, int t, int n, uint32_t* buf,
                                                int rw) {
  copy_in(buf, rows + (int64_t)t * rw, n * rw);
}

__device__ __forceinline__ void stage_groups(const JobDev& J, const UnitLds& u) {
  const int n_grp = J.n_pad >> 2;
  const GLOBAL_AS int32_t* grp = gconst(J.grp);
  const GLOBAL_AS int32_t* gbase = gconst(J.gbase);
  const GLOBAL_AS uint32_t* gdeg = gconst(J.gdeg);
  const int nt = (int)blockDim.x;
  for (int i0 = (int)threadIdx.x; i0 < n_grp; i0 += 4 * nt) {
    int32_t a[4], b[4];
    uint32_t c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = min(i0 + k * nt, n_grp - 1);
      a[k] = grp[i];
      b[k] = gbase[i];
      c[k] = gdeg[i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (i0 + k * nt < n_grp) {
        u.gword[i0 + k * nt] = a[k];
        u.gbase[i0 + k * nt] = b[k];
        u.gdeg[i0 + k * nt] = c[k];
      }
  }
}

__device__ __forceinline__ int next_unit(const int32_t* list_off, int32_t* ctr, int& tried) {
  const int home = blockIdx.x & 7;
  if (tried == 0) {
    const int i = atomicAdd(&ctr[home], 1);
    if (list_off[home] + i < list_off[home + 1]) return list_off[home] + i;
    tried = 1;
  }
  // The other lists' cursors, read together: a cursor that has passed its
  // list's end stays there (cursors only grow), so such a list needs no
  // claim.  At the end of a launch this costs one memory round trip instead
  // of one atomic per list.
  int c[7];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    c[k - 1] = __hip_atomic_load(&ctr[(home + k) & 7], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (; tried < 8; ++tried) {
    const int L = (home + tried) & 7;
    int seen = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) seen = k == tried ? c[k - 1] : seen;
    if (list_off[L] + seen >= list_off[L + 1]) continue;
    const int i = atomicAdd(&ctr[L], 1);
    if (list_off[L] + i < list_off[L + 1]) return list_off[L] + i;
  }
  return -1;
}

// Flip pushes of one group: flipped slot j adds (-2 w s_new) << 1 to the
// packed word of each neighbour.  Entries are taken four at a time; indices
// past the slot's degree repeat its last entry and add zero, so the inner
// body has no per-entry branch.
// The same with the first four entries of every slot already fetched
// (q[j][i] = aw[o[j] + i]); only slots of degree above four load more.
__device__ __forceinline__ void push_group_prefetched(int32_t* st, const GLOBAL_AS i32x2* __restrict__ aw,
                                                      const int (&o)[4], uint32_t dg, uint32_t fm,
                                                      const int (&w)[4], const i32x2 (&q)[4][4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int d = (int)((dg >> (8 * j)) & 255u);
    if ((fm >> j) & 1u) {
      const int sgn4 = (w[j] & 1) ? -4 : 4;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < d) atomicAdd(&st[q[j][i].x], sgn4 * q[j][i].y);
      for (int e0 = 4; e0 < d; e0 += 4) {
        i32x2 r[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = aw[o[j] + min(e0 + i, d - 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(&st[r[i].x], e0 + i < d ? sgn4 * r[i].y : 0);
      }
    }
  }
}

// Pushes of one flipped vertex described by a flip-list entry:
// bits 0..16 = first adjacency entry, 17..24 = degree, 25 = new spin is +1.
__device__ __forceinline__ void push_entry(int32_t* st, const uint16_t* adj16, uint32_t e) {
  const int o = (int)(e & 0x1FFFFu);
  const int d = (int)((e >> 17) & 255u);
  const int sgn4 = ((e >> 25) & 1u) ? -4 : 4;
  if (d == 4 && (o & 3) == 0) {
    const uint2 e4 = *reinterpret_cast<const uint2*>(adj16 + o);
    const uint32_t a0 = e4.x & 0xFFFFu, a1 = e4.x >> 16, a2 = e4.y & 0xFFFFu, a3 = e4.y >> 16;
    atomicAdd(&st[a0 >> 1], (a0 & 1u) ? sgn4 : -sgn4);
    atomicAdd(&st[a1 >> 1], (a1 & 1u) ? sgn4 : -sgn4);
    atomicAdd(&st[a2 >> 1], (a2 & 1u) ? sgn4 : -sgn4);
    atomicAdd(&st[a3 >> 1], (a3 & 1u) ? sgn4 : -sgn4);
  } else {
    for (int i = 0; i < d; ++i) {
      const uint32_t a = adj16[o + i];
      atomicAdd(&st[a >> 1], (a & 1u) ? sgn4 : -sgn4);
    }
  }
}

// The flipped vertices of a wave's groups are appended to the wave's list
// (ballot + rank among set lanes) and then pushed with every active lane
// taking one entry per round, instead of four mostly-masked slot passes.
__device__ __forceinline__ void push_wave_compacted(int32_t* st, const uint16_t* adj16,
                                                    uint32_t* list, int base, uint32_t dg,
                                                    uint32_t fm, const int (&w)[4]) {
  const uint64_t active = __ballot(1);
  const uint32_t lo = (uint32_t)active, hi = (uint32_t)(active >> 32);
  const int arank = (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
  const int nact = __popcll(active);
  int n = 0;
  int o = base;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int d = (int)((dg >> (8 * j)) & 255u);
    const bool f = (fm >> j) & 1u;
    const uint64_t m = __ballot(f);
    if (f) {
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      list[n + rank] = (uint32_t)o | ((uint32_t)d << 17) | ((uint32_t)(w[j] & 1) << 25);
    }
    n += __popcll(m);
    o += d;
  }
  for (int b = 0; b < n; b += nact) {
    const int i = b + arank;
    if (i < n) push_entry(st, adj16, list[i]);
  }
}

// Degree-4 (bond) pushes.  A flip of v changes the bond bit of each of its
// edges, and neighbour u holds that bit at position kBondShift + (e XOR 1)
// when u is entry e of v (the host labels edges that way), so a push is an
// LDS XOR of a mask fixed by e.  The LDS byte address is one 16 x 16 + 32
// multiply-add of the entry's 16-bit word index (low or high half of the
// word), written out because the compiler extracts the halves separately.
typedef __attribute__((address_space(3))) int32_t lds_i32;

template <int HI>
__device__ __forceinline__ uint32_t lds_byte_addr(uint32_t two, uint32_t base) {
  uint32_t a;
  if (HI)
    asm("v_mad_u32_u16 %0, %1, 4, %2 op_sel:[1,0,0,0]" : "=v"(a) : "v"(two), "v"(base));
  else
    asm("v_mad_u32_u16 %0, %1, 4, %2" : "=v"(a) : "v"(two), "v"(base));
  return a;
}

// The four pushes of one slot; lo and hi hold its entries 0, 1 and 2, 3.
__device__ __forceinline__ void push_bond_slot(uint32_t base, uint32_t lo, uint32_t hi) {
  __hip_atomic_fetch_xor((lds_i32*)(uintptr_t)lds_byte_addr<0>(lo, base), 1 << (kBondShift + 1),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_xor((lds_i32*)(uintptr_t)lds_byte_addr<1>(lo, base), 1 << kBondShift,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_xor((lds_i32*)(uintptr_t)lds_byte_addr<0>(hi, base), 1 << (kBondShift + 3),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __hip_atomic_fetch_xor((lds_i32*)(uintptr_t)lds_byte_addr<1>(hi, base), 1 << (kBondShift + 2),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Test key of a packed word w = (h << 1) | b (spin s = 2 b - 1), with
// k = s h the quantity the acceptance test compares (the energy moves by
// 2 k): x = 2 k - c, where c = 1 - b.  For b = 1, x = w XOR 1 = 2 h; for
// b = 0, x = NOT w = -2 h - 1.  So x = w XNOR (m AND -2) with m = -b: one
// bit-field extract and one three-input logic operation.  x <= 2 len holds
// exactly when k <= len, and entry x of a row (rows of 2 kw + 2 words)
// holds the threshold of k = ceil(x / 2).  Written out because the
// compiler turns the select into longer sequences.
__device__ __forceinline__ int field_key(int w, int& m) {
  int x;
  asm("v_bfe_i32 %0, %1, 0, 1" : "=v"(m) : "v"(w));
  asm("v_bitop3_b32 %0, %1, %2, -2 bitop3:0x87" : "=v"(x) : "v"(w), "v"(m));
  return x;
}

// Row entry of key x: x clamped to [0, 2 kw] by one median-of-three.
__device__ __forceinline__ int clamp_row_index(int x, int kw2) {
  int i;
  asm("v_med3_i32 %0, %1, 0, %2" : "=v"(i) : "v"(x), "s"(kw2));
  return i;
}

template <int BLOCK, int ADJ>
__device__ void field_unit(const JobDev& J, const int block, int32_t* smem, FieldShared& sh) {
  const int G = J.G;
  const int TPR = BLOCK / G;  // threads per replica, a multiple of 64
  const int tid = threadIdx.x;
  const int rl = tid / TPR, lt = tid - rl * TPR;
  const int r = block * G + rl;
  const bool live = r < J.R;
  const int n_pad = J.n_pad, n_grp = n_pad >> 2;
  const int SW = field_state_words(n_pad);
  int32_t* st = smem + rl * SW;
  // Word of slot j of group g.  The degree-4 forms keep the state in tiles
  // of 64 groups with a plane per slot, so that per-slot accesses of
  // consecutive groups (the spin flips, and the pushes, whose neighbours
  // are consecutive groups of another class) hit consecutive LDS banks and
  // a group's four words are constant offsets (256 bytes) apart; the other
  // forms keep a group's four words together.
  constexpr bool SOA = ADJ == kAdjLdsDeg4 || ADJ == kAdjHbmDeg4;
  auto widx = [&](int g, int j) { return SOA ? tile_word(g, j) : 4 * g + j; };
  const int C = J.n_colours;
  // row words: the degree-4 forms test a bond count, the others the key
  // of field_key
  const int RW = SOA ? kBondRowWords : 2 * J.kw + 2;
  const uint32_t* const rows = SOA ? J.tqb : J.tqp;
  UnitLds U = unit_lds(reinterpret_cast<uint32_t*>(smem), G * SW, J.row_chunk * RW, 2 * C, n_grp);
  const uint32_t k0 = J.seed_lo, k1 = J.seed_hi;
  const int W = J.W;
  const GLOBAL_AS i32x2* __restrict__ aw = gconst(reinterpret_cast<const i32x2*>(J.aw));

  if (tid < 4 * kMaxReplicasPerBlock) (&sh.eacc[0][0])[tid] = 0;
  if (tid < kMaxReplicasPerBlock) sh.nacc[tid] = 0;

  // ---- state in: initial draw, or the words saved by the previous chunk
  const bool fresh = J.t_begin == 0;
  auto put_group = [&](int g, const int4& w4) {
    if (SOA) {
      st[widx(g, 0)] = w4.x;
      st[widx(g, 1)] = w4.y;
      st[widx(g, 2)] = w4.z;
      st[widx(g, 3)] = w4.w;
    } else {
      *reinterpret_cast<int4*>(st + 4 * g) = w4;
    }
  };
  // a resumed chunk's per-replica scalars, loaded with its state
  int E_in = 0, best_cut_in = 0, best_sweep_in = 0;
  unsigned long long acc_in = 0;
  if (live && !fresh) {
    E_in = J.energy[r];
    best_cut_in = J.best_cut[r];
    best_sweep_in = J.best_sweep[r];
    acc_in = J.accepts[r];
  }
  if (live && !fresh) {
    // four loads of each lane in flight at a time
    const GLOBAL_AS u32x4* sv = gconst(reinterpret_cast<const u32x4*>(J.save + (int64_t)r * n_pad));
    for (int g0 = lt; g0 < n_grp; g0 += 4 * TPR) {
      u32x4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = sv[min(g0 + k * TPR, n_grp - 1)];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (g0 + k * TPR < n_grp)
          put_group(g0 + k * TPR, make_int4((int)v[k].x, (int)v[k].y, (int)v[k].z, (int)v[k].w));
    }
  }
  if (live && fresh) {
    for (int g = lt; g < n_grp; g += TPR) {
      int4 w4;
      if (fresh) {
        const int gw = J.grp[g];
        const int cnt = (gw >> kGroupCountShift) + 1;
        uint32_t bits;
        if (J.flags & kJobInitGiven) {
          bits = 0;
          for (int j = 0; j < cnt; ++j)
            bits |= (J.init_spins[(int64_t)r * n_pad + 4 * g + j] > 0 ? 1u : 0u) << j;
        } else {
          const uint4 x = group_block((uint32_t)g, 0, r, kTagInit, k0, k1);
          bits = (x.x >> 31) | ((x.y >> 31) << 1) | ((x.z >> 31) << 2) | ((x.w >> 31) << 3);
        }
        w4.x = (int)(bits & 1u);
        w4.y = cnt > 1 ? (int)((bits >> 1) & 1u) : kPadWord;
        w4.z = cnt > 2 ? (int)((bits >> 2) & 1u) : kPadWord;
        w4.w = cnt > 3 ? (int)((bits >> 3) & 1u) : kPadWord;
      }
      put_group(g, w4);
    }
  }
  // Parallel tempering: replica rl's row is its temperature's for the
  // whole launch (the exchanges happen between launches), staged once at
  // U.tq + rl RW; the chunk is never restaged.
  const bool pt = J.temp != nullptr;
  const int CH = pt ? 0x7FFFFFFF : J.row_chunk;
  if (pt) {
    for (int i = tid; i < G * RW; i += BLOCK) {
      const int q = i / RW, rq = block * G + q;
      U.tq[i] = rq < J.R ? rows[(int64_t)J.temp[rq] * RW + (i - q * RW)] : 0u;
    }
  } else {
    stage_row_chunk(rows, J.t_begin, min(CH, J.t_end - J.t_begin), U.tq, RW);
  }
  copy_in(U.cls, J.cls, 2 * C);
  stage_groups(J, U);
  if (ADJ == kAdjLds) {
    stage_adjacency(J, U);
    place_flip_lists(U, J.M);
  } else if (ADJ == kAdjLdsDeg4) {
    stage_adjacency_deg4(J, U);
  }
  uint32_t* flist = ADJ == kAdjLds ? U.flips + (threadIdx.x >> 6) * 256 : nullptr;
  // LDS byte addresses of this replica's words and of the degree-4 blocks
  const uint32_t st_base = (uint32_t)(uintptr_t)(lds_i32*)st;
  const uint32_t blk_base = (uint32_t)(uintptr_t)(lds_i32*)U.adj16;
  __syncthreads();

  int E, best_cut, best_sweep;
  bool snap;
  // a resumed tempering segment may have its bond words saved as they were
  const bool bond_in = SOA && !fresh && (J.flags & kJobLoadBond);
  if (SOA && !bond_in) {
    // Bond words from the spins (bit 0 of every word at this point), for a
    // fresh start and a resumed chunk alike.  Only bit 0 of other words is
    // read while words are rewritten, and bit 0 keeps the spin.
    int part = 0;
    if (live) {
      for (int p = lt; p < n_pad; p += TPR) {
        const int g = p >> 2, j = p & 3;
        int32_t* wp = st + tile_word(g, j);
        if (j > (U.gword[g] >> kGroupCountShift)) {
          *wp = kBondPadWord;
          continue;
        }
        // the slot's two entry words and the weight-sign word of the block
        uint32_t lo, hi, signs;
        if (ADJ == kAdjLdsDeg4) {
          const uint32_t* b = reinterpret_cast<const uint32_t*>(U.adj16) + kDeg4BlockWords * g;
          lo = b[2 * j];
          hi = b[2 * j + 1];
          signs = b[9];
        } else {
          const GLOBAL_AS uint32_t* b =
              gconst(reinterpret_cast<const uint32_t*>(J.adj4)) + kDeg4BlockWords * (int64_t)g;
          lo = b[2 * j];
          hi = b[2 * j + 1];
          signs = b[9];
        }
        const uint32_t bv = (uint32_t)*wp & 1u;
        uint32_t word = bv | ((bv ^ 1u) << 1);
        for (int e = 0; e < 4; ++e) {
          const uint32_t nw = ((e < 2 ? lo : hi) >> (16 * (e & 1))) & 0xFFFFu;
          const uint32_t bu = (uint32_t)st[nw] & 1u;
          const uint32_t wpos = (signs >> (4 * j + e)) & 1u;
          word |= (1u ^ bv ^ bu ^ wpos) << (kBondShift + e);
        }
        part += 2 * __popc(word) - 6;  // k = s h
        *wp = (int32_t)word;
      }
    }
    __syncthreads();
    if (fresh) {
      part = wave_sum(part);
      if ((tid & 63) == 0 && part != 0) atomicAdd(&sh.eacc[3][rl], part);
      __syncthreads();
      E = -sh.eacc[3][rl] / 2;
    }
  }
  if (fresh && SOA) {
    best_cut = (W - E) / 2;
    best_sweep = -1;
    snap = true;  // the initial state is written during sweep 0
  } else if (fresh) {
    // fields from scratch: h_p = -sum_q w_pq s_q.  Only bit 0 of other
    // words is read while fields are written, and that bit is unchanged.
    int part = 0;
    if (live) {
      for (int p = lt; p < n_pad; p += TPR) {
        const int g = p >> 2, j = p & 3;
        if (j > (U.gword[g] >> kGroupCountShift)) continue;  // padding keeps kPadWord
        const uint32_t dg = U.gdeg[g];
        int a = U.gbase[g];
        for (int i = 0; i < j; ++i) a += (int)((dg >> (8 * i)) & 255u);
        const int d = (int)((dg >> (8 * j)) & 255u);
        // local fields: h starts at 2 b, and the energy sum takes h + 2 b
        const int bf = J.bfield ? 2 * J.bfield[p] : 0;
        int h = bf;
        for (int e = 0; e < d; ++e) {
          const i32x2 q = aw[a + e];
          h -= q.y * ((st[widx(q.x >> 2, q.x & 3)] & 1) ? 1 : -1);
        }
        const int b = st[widx(g, j)] & 1;
        st[widx(g, j)] = (h << 1) | b;
        part += b ? h + bf : -(h + bf);
      }
    }
    part = wave_sum(part);
    if ((tid & 63) == 0 && part != 0) atomicAdd(&sh.eacc[3][rl], part);
    __syncthreads();
    E = -sh.eacc[3][rl] / 2;
    best_cut = (W - E) / 2;
    best_sweep = -1;
    snap = true;  // the initial state is written during sweep 0
  } else {
    E = E_in;
    best_cut = best_cut_in;
    best_sweep = best_sweep_in;
    snap = false;
  }

  GLOBAL_AS int8_t* best = gmut(static_cast<int8_t*>(J.best)) + (int64_t)r * n_pad;
  const int kw2 = 2 * J.kw;
  // sum over this lane's accepted flips of x + m = 2 k - 1; the sweep's
  // energy change adds the wave's accepted count
  int dk = 0;
  int nacc = 0;       // accepted flips of this wave (wave-uniform)
  int nacc_mark = 0;  // nacc at the start of the sweep
  // Class bounds (at most kMaxFieldColours classes): lane i of two
  // registers keeps words i and 64 + i, and a pass takes its bounds with
  // lane reads, so no LDS wait sits at the start of a pass.
  const int cls_a = (tid & 63) < 2 * C ? U.cls[tid & 63] : 0;
  const int cls_b = 64 + (tid & 63) < 2 * C ? U.cls[64 + (tid & 63)] : 0;
  auto bound = [&](int i) {
    const int a = __builtin_amdgcn_readlane(cls_a, i & 63), b = __builtin_amdgcn_readlane(cls_b, i & 63);
    return i < 64 ? a : b;
  };
  // Rows come in chunks of CH sweeps, one HBM copy and barrier per chunk,
  // so that the passes themselves issue no HBM loads: a wait for one would
  // also wait for the snapshot stores still in flight.
  int tc = 0;  // sweep within the staged chunk
  // The row's bound: twice the largest acceptable k (key rows), or the
  // largest acceptable bond count plus one (degree-4 rows).  The next
  // sweep's is read during the last pass, so no LDS read is pending when a
  // sweep starts.
  const int row_of_replica = pt ? rl : 0;
  int len2_next = (int)U.tq[row_of_replica * RW + RW - 1];
  for (int t = J.t_begin; t < J.t_end; ++t) {
    if (tc == CH) {
      stage_row_chunk(rows, t, min(CH, J.t_end - t), U.tq, RW);
      tc = 0;
      __syncthreads();
      len2_next = (int)U.tq[RW - 1];
    }
    const uint32_t* row = U.tq + (pt ? row_of_replica : tc) * RW;
    const int len2 = len2_next;
    ++tc;
    for (int c = 0; c < C; ++c) {
      const int g0 = bound(2 * c), g1 = bound(2 * c + 1);
      if (live) {
        for (int gi = g0 + lt; gi < g1; gi += TPR) {
          // Addresses are formed from the group index in each iteration:
          // most lanes run one iteration per pass, and a separate induction
          // variable per array (the compiler's default) costs more.
          int g = gi;
          asm("" : "+v"(g));
          // byte address of the group's slot-0 word in the tiled layout:
          // 4 tile_word(g, 0) = 4 g + 12 (g AND -64)
          lds_i32* const s0 =
              (lds_i32*)(uintptr_t)(st_base + ((uint32_t)g << 2) + __umul24((uint32_t)g & ~63u, 12u));
          int4 w4;
          if (SOA) {
            w4.x = s0[0];
            w4.y = s0[64];
            w4.z = s0[128];
            w4.w = s0[192];
          } else {
            w4 = *reinterpret_cast<const int4*>(st + 4 * g);
          }
          // degree-4 forms: the group's neighbour entries are fetched with
          // its state
          uint4 a01 = make_uint4(0u, 0u, 0u, 0u), a23 = a01;
          if (ADJ == kAdjLdsDeg4) {
            typedef __attribute__((address_space(3))) const u32x4 lds_u32x4;
            lds_u32x4* blk = (lds_u32x4*)(uintptr_t)(blk_base + __umul24((uint32_t)g, 48u));
            const u32x4 b0 = blk[0], b1 = blk[1];
            a01 = make_uint4(b0.x, b0.y, b0.z, b0.w);
            a23 = make_uint4(b1.x, b1.y, b1.z, b1.w);
          } else if (ADJ == kAdjHbmDeg4) {
            const GLOBAL_AS u32x4* blk = gconst(reinterpret_cast<const u32x4*>(J.adj4)) + 3 * g;
            const u32x4 b0 = blk[0], b1 = blk[1];
            a01 = make_uint4(b0.x, b0.y, b0.z, b0.w);
            a23 = make_uint4(b1.x, b1.y, b1.z, b1.w);
          }
          // {position, w} form: the first four entries of every slot are
          // fetched with the state, so that a flip's pushes do not wait for
          // HBM; entries past a slot's degree (the next slot's, or the
          // array's zero padding) are not used
          int o[4] = {0, 0, 0, 0};
          uint32_t dg = 0;
          i32x2 q[4][4];
          if (ADJ == kAdjHbm) {
            dg = U.gdeg[g];
            int base = U.gbase[g];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              o[j] = base;
              base += (int)((dg >> (8 * j)) & 255u);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
              for (int i = 0; i < 4; ++i) q[j][i] = aw[o[j] + i];
          }
          // all of the group's reads go out before any arithmetic
          __builtin_amdgcn_sched_barrier(0);
          int w[4] = {w4.x, w4.y, w4.z, w4.w};
          // Lazy best-state snapshot of this group (its end-of-previous-sweep
          // spins).  The degree-4 forms keep w unchanged in registers and
          // take it at the end of the iteration, so that no branch separates
          // the group's loads from their first use.
          auto snapshot = [&]() {
            const uint32_t bits = (w[0] & 1) | ((w[1] & 1) << 1) | ((w[2] & 1) << 2) | ((w[3] & 1) << 3);
            *reinterpret_cast<GLOBAL_AS uint32_t*>(best + 4 * g) = spins_to_bytes(bits);
          };
          if (!SOA && snap) snapshot();
          // Row entry 0 accepts k <= 0 and k above the row's length is
          // refused by the length test (padding slots have the key
          // 2^31 - 2, or a bond count above every bound), so each slot's
          // test is two comparisons.
          // k: the bond count plus one (degree-4 forms, rows indexed by
          // it directly) or field_key; m = -(spin bit)
          int k[4], m[4];
          uint32_t thr[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (SOA)
              k[j] = __popc((uint32_t)w[j]);
            else
              k[j] = field_key(w[j], m[j]);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) thr[j] = row[SOA ? k[j] : clamp_row_index(k[j], kw2)];
          // Nearly every group needs its Philox block, so it is drawn
          // unconditionally, after the threshold reads are issued: its
          // arithmetic covers their latency.
          __builtin_amdgcn_sched_barrier(0);
          const uint4 x = group_block((uint32_t)g, t, r, kTagSweep, k0, k1);
          bool acc[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bool in_row = k[j] <= len2, below = pick(x, j) <= thr[j];
            acc[j] = in_row & below;
            // two ballots of comparisons: their masks are ANDed as scalars
            nacc += __popcll(__ballot(in_row) & __ballot(below));
          }
          if (ADJ == kAdjLdsDeg4 || ADJ == kAdjHbmDeg4) {
            // Within a pass only the owning lane touches a group's own
            // words (neighbours are in other classes and do not flip), so
            // a flip is a plain LDS store of the word with its spin pair
            // and four bond bits inverted; each push is an LDS XOR of one
            // bond bit of a neighbour's word, which several flips of the
            // pass may change.
            const uint32_t e[8] = {a01.x, a01.y, a01.z, a01.w, a23.x, a23.y, a23.z, a23.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (acc[j]) {
                s0[64 * j] = w[j] ^ kBondFlipMask;
                dk += k[j];
                push_bond_slot(st_base, e[2 * j], e[2 * j + 1]);
              }
            }
            if (snap) snapshot();
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              w[j] = acc[j] ? w[j] ^ 1 : w[j];
              dk += acc[j] ? k[j] + m[j] : 0;
            }
            const bool any = acc[0] | acc[1] | acc[2] | acc[3];
            if (any) *reinterpret_cast<int4*>(st + 4 * g) = make_int4(w[0], w[1], w[2], w[3]);
            const uint32_t fm =
                (acc[0] ? 1u : 0u) | (acc[1] ? 2u : 0u) | (acc[2] ? 4u : 0u) | (acc[3] ? 8u : 0u);
            if (ADJ == kAdjLds)
              push_wave_compacted(st, U.adj16, flist, U.gbase[g], U.gdeg[g], fm, w);
            else if (any)
              push_group_prefetched(st, aw, o, dg, fm, w, q);
          }
        }
      }
      if (c == C - 1) {
        // degree-4 forms: 2 k = 4 (bond count + 1) - 12; others:
        // 2 k = (x + m) + 1
        const int s = SOA ? 4 * wave_sum(dk) - 12 * (nacc - nacc_mark)
                          : wave_sum(dk) + (nacc - nacc_mark);
        if ((tid & 63) == 0 && s != 0) atomicAdd(&sh.eacc[t % 3][rl], s);
        dk = 0;
        nacc_mark = nacc;
        if (tc < CH) len2_next = (int)U.tq[(pt ? row_of_replica : tc) * RW + RW - 1];
      }
      __syncthreads();
    }
    E += sh.eacc[t % 3][rl];
    if (lt == 0) sh.eacc[(t + 2) % 3][rl] = 0;
    const int cut = (W - E) / 2;
    snap = cut > best_cut;
    if (snap) {
      best_cut = cut;
      best_sweep = t;
    }
    if ((J.flags & kJobTrace) && lt == 0 && live) J.trace[(int64_t)t * J.R + r] = E;
  }

  // ---- state out
  if (live) {
    for (int g = lt; g < n_grp; g += TPR) {
      int4 w4;
      if (SOA && (J.flags & kJobSaveBond)) {
        // the next segment reads the bond words back as they are
        w4 = make_int4(st[widx(g, 0)], st[widx(g, 1)], st[widx(g, 2)], st[widx(g, 3)]);
      } else if (SOA) {
        // bond words back to packed fields: k = 2 popc - 6, h = s k
        int v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int x = st[widx(g, j)];
          const int b = x & 1, kk = 2 * __popc((uint32_t)x) - 6;
          v[j] = x == kBondPadWord ? kPadWord : (((b ? kk : -kk) << 1) | b);
        }
        w4 = make_int4(v[0], v[1], v[2], v[3]);
      } else {
        w4 = *reinterpret_cast<const int4*>(st + 4 * g);
      }
      if (snap) {
        const uint32_t bits = (w4.x & 1) | ((w4.y & 1) << 1) | ((w4.z & 1) << 2) | ((w4.w & 1) << 3);
        *reinterpret_cast<GLOBAL_AS uint32_t*>(best + 4 * g) = spins_to_bytes(bits);
      }
      // a run that keeps no state for later reads (J.save null) skips it
      if (J.save) *reinterpret_cast<int4*>(J.save + (int64_t)r * n_pad + 4 * g) = w4;
    }
  }
  // lane 0 takes part in every group iteration of its wave, so its count
  // is the wave's
  if ((tid & 63) == 0 && nacc != 0) atomicAdd(&sh.nacc[rl], nacc);
  __syncthreads();
  if (lt == 0 && live) {
    J.accepts[r] = acc_in + (unsigned long long)sh.nacc[rl];
    J.energy[r] = E;
    J.best_cut[r] = best_cut;
    J.best_sweep[r] = best_sweep;
  }
}

template <int BLOCK, int ADJ>
__global__ void __launch_bounds__(BLOCK)
k_field(const JobDev* __restrict__ jobs, const int2* __restrict__ units,
        const int32_t* __restrict__ list_off, int32_t* __restrict__ ctr) {
  extern __shared__ __align__(16) int32_t smem[];
  __shared__ FieldShared sh;
  int tried = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh.unit = next_unit(list_off, ctr, tried);
    __syncthreads();
    const int u = sh.unit;
    if (u < 0) break;
    const int2 un = units[u];
    const JobDev J = jobs[un.x];  // by value: fields stay in registers
    if (ADJ != kAdjPerJob) {
      field_unit<BLOCK, ADJ>(J, un.y, smem, sh);
    } else if (J.adj_form == kAdjLdsDeg4) {
      field_unit<BLOCK, kAdjLdsDeg4>(J, un.y, smem, sh);
    } else if (J.adj_form == kAdjLds) {
      field_unit<BLOCK, kAdjLds>(J, un.y, smem, sh);
    } else if (J.adj_form == kAdjHbmDeg4) {
      field_unit<BLOCK, kAdjHbmDeg4>(J, un.y, smem, sh);
    } else {
      field_unit<BLOCK, kAdjHbm>(J, un.y, smem, sh);
    }
  }
}

// ================================================================ msc
// Unit = (job, block of G words); word w holds replicas 32w .. 32w+31.

struct MscShared {
  int32_t unit;
  int32_t eacc[4][kMaxWordsPerBlock * 32];
  int32_t E[kMaxWordsPerBlock * 32];
  int32_t best_cut[kMaxWordsPerBlock * 32];
  int32_t best_sweep[kMaxWordsPerBlock * 32];
  uint32_t snap[kMaxWordsPerBlock];
};

constexpr int kMscPlanes = 5;  // degree <= 31

// Add the 32 one-bit values of x into the bit-sliced counter U.
__device__ __forceinline__ void slice_add(uint32_t (&U)[kMscPlanes], uint32_t x, int planes) {
#pragma unroll
  for (int b = 0; b < kMscPlanes; ++b) {
    if (b < planes) {
      const uint32_t c = U[b] & x;
      U[b] ^= x;
      x = c;
    }
  }
}

__device__ __forceinline__ int slice_get(const uint32_t (&U)[kMscPlanes], int bit, int planes) {
  int u = 0;
#pragma unroll
  for (int b = 0; b < kMscPlanes; ++b)
    if (b < planes) u |= (int)((U[b] >> bit) & 1u) << b;
  return u;
}

// Lane layout inside a word slice: four lanes per group ("quad"), lane o of
// the quad decides replicas 8o .. 8o+7 of the word; the four partial flip
// masks are OR-combined with lane shuffles.
__device__ __forceinline__ uint32_t quad_or(uint32_t v) {
  v |= (uint32_t)__shfl_xor((int)v, 1, 64);
  v |= (uint32_t)__shfl_xor((int)v, 2, 64);
  return v;
}

// Sum over the lanes of a wave that share (lane & 3).
__device__ __forceinline__ int quad_lane_sum(int v) {
#pragma unroll
  for (int off = 32; off >= 4; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Unsatisfied-bond counters of the four slots of a group: bit r of slice b
// of U[j] is bit b of the number of bonds of slot j that replica r leaves
// unsatisfied (w s_i s_j = +1).  Adjacency entries are loaded before use.
__device__ __forceinline__ void group_unsat(const uint32_t* st, const GLOBAL_AS uint32_t* __restrict__ adjm,
                                            int base, uint32_t dg, int cnt, const uint32_t (&S)[4],
                                            uint32_t (&U)[4][kMscPlanes], int (&d)[4], int planes) {
  int o[4];
  int acc = base;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    d[j] = j < cnt ? (int)((dg >> (8 * j)) & 255u) : 0;
    o[j] = acc;
    acc += (int)((dg >> (8 * j)) & 255u);
#pragma unroll
    for (int b = 0; b < kMscPlanes; ++b) U[j][b] = 0;
  }
  uint32_t q[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < d[j]) q[j][e] = adjm[o[j] + e];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (e < d[j]) slice_add(U[j], S[j] ^ st[q[j][e] >> 1] ^ ((q[j][e] & 1u) ? 0xFFFFFFFFu : 0u), planes);
    for (int e = 4; e < d[j]; ++e) {
      const uint32_t am = adjm[o[j] + e];
      slice_add(U[j], S[j] ^ st[am >> 1] ^ ((am & 1u) ? 0xFFFFFFFFu : 0u), planes);
    }
  }
}

template <int BLOCK>
__device__ void msc_unit(const JobDev& J, const int block, uint32_t* smem, MscShared& sh,
                         const int planes) {
  const int Gw = J.G;
  const int TPR = BLOCK / Gw;
  const int QPR = TPR >> 2;  // quads per word slice
  const int tid = threadIdx.x;
  const int wl = tid / TPR, lt = tid - wl * TPR;
  const int o = lt & 3, gq = lt >> 2;
  const int wi = block * Gw + wl;
  const int r0 = 32 * wi;
  const int rb = r0 + 8 * o;  // first replica decided by this lane
  const bool live = r0 < J.R;
  const int n_pad = J.n_pad, n_grp = n_pad >> 2;
  uint32_t* st = smem + wl * n_pad;
  const UnitLds U = unit_lds(smem, Gw * n_pad, 2 * J.kw, 0, n_grp);
  const uint32_t k0 = J.seed_lo, k1 = J.seed_hi;
  const int C = J.n_colours;
  const int W = J.W;
  const bool fresh = J.t_begin == 0;
  const GLOBAL_AS uint32_t* __restrict__ adjm = gconst(J.adjm);

  for (int i = tid; i < 4 * kMaxWordsPerBlock * 32; i += BLOCK) (&sh.eacc[0][0])[i] = 0;

  if (live) {
    for (int g = gq; g < n_grp; g += QPR) {
      uint32_t b[4] = {0, 0, 0, 0};
      const int gw = J.grp[g];
      const int cnt = (gw >> kGroupCountShift) + 1;
      if (fresh) {
        if (J.flags & kJobInitGiven) {
          for (int i = 0; i < 8; ++i) {
            const int r = rb + i;
            if (r < J.R)
              for (int j = 0; j < cnt; ++j)
                b[j] |= (J.init_spins[(int64_t)r * n_pad + 4 * g + j] > 0 ? 1u : 0u) << (8 * o + i);
          }
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const uint4 x = group_block((uint32_t)g, 0, rb + i, kTagInit, k0, k1);
            b[0] |= (x.x >> 31) << (8 * o + i);
            b[1] |= (x.y >> 31) << (8 * o + i);
            b[2] |= (x.z >> 31) << (8 * o + i);
            b[3] |= (x.w >> 31) << (8 * o + i);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = j < cnt ? quad_or(b[j]) : 0u;
        if (o == 0) *reinterpret_cast<uint4*>(st + 4 * g) = make_uint4(b[0], b[1], b[2], b[3]);
      } else if (o == 0) {
        *reinterpret_cast<uint4*>(st + 4 * g) = *reinterpret_cast<const uint4*>(
            reinterpret_cast<const uint32_t*>(J.save) + (int64_t)wi * n_pad + 4 * g);
      }
    }
  }
  stage_row(J, J.t_begin, U.tq);
  stage_groups(J, U);
  __syncthreads();

  GLOBAL_AS uint32_t* bestw = gmut(static_cast<uint32_t*>(J.best)) + (int64_t)wi * n_pad;
  if (fresh) {
    // E_r = sum_p u_{p,r} - M, with u the unsatisfied bonds at p.
    int cnt8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (live) {
      for (int g = gq; g < n_grp; g += QPR) {
        const int cnt = (U.gword[g] >> kGroupCountShift) + 1;
        const uint4 s4 = *reinterpret_cast<const uint4*>(st + 4 * g);
        const uint32_t S[4] = {s4.x, s4.y, s4.z, s4.w};
        uint32_t Uq[4][kMscPlanes];
        int d[4];
        group_unsat(st, adjm, U.gbase[g], U.gdeg[g], cnt, S, Uq, d, planes);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int i = 0; i < 8; ++i) cnt8[i] += slice_get(Uq[j], 8 * o + i, planes);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int s = quad_lane_sum(cnt8[i]);
      if ((tid & 63) < 4 && s != 0) atomicAdd(&sh.eacc[3][wl * 32 + 8 * o + i], s);
    }
    __syncthreads();
    if (lt < 32) {
      const int e = sh.eacc[3][wl * 32 + lt] - J.M;
      sh.E[wl * 32 + lt] = e;
      sh.best_cut[wl * 32 + lt] = (W - e) / 2;
      sh.best_sweep[wl * 32 + lt] = -1;
    }
    if (lt == 0) sh.snap[wl] = 0xFFFFFFFFu;
  } else {
    if (lt < 32) {
      const int r = r0 + lt;
      sh.E[wl * 32 + lt] = r < J.R ? J.energy[r] : 0;
      sh.best_cut[wl * 32 + lt] = r < J.R ? J.best_cut[r] : 0;
      sh.best_sweep[wl * 32 + lt] = r < J.R ? J.best_sweep[r] : 0;
    }
    if (lt == 0) sh.snap[wl] = 0;
  }
  __syncthreads();

  int dE[8], nacc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    dE[i] = 0;
    nacc[i] = 0;
  }

  for (int t = J.t_begin; t < J.t_end; ++t) {
    const int len = gconst(J.tq_len)[t];
    const uint32_t* row = U.tq + (t & 1) * J.kw;
    const uint32_t snapm = sh.snap[wl];
    const bool draw_needed = len > 0;  // otherwise no move with k > 0 can pass
    for (int c = 0; c < C; ++c) {
      if (c == C - 1) stage_row(J, t + 1, U.tq);
      const int g0 = gconst(J.cls)[2 * c], g1 = gconst(J.cls)[2 * c + 1];
      if (live) {
        for (int g = g0 + gq; g < g1; g += QPR) {
          const int gw = U.gword[g];
          const int cnt = (gw >> kGroupCountShift) + 1;
          const uint4 s4 = *reinterpret_cast<const uint4*>(st + 4 * g);
          const uint32_t S[4] = {s4.x, s4.y, s4.z, s4.w};
          if (snapm && o == 0) {
            u32x4 b4 = *reinterpret_cast<const GLOBAL_AS u32x4*>(bestw + 4 * g);
            b4.x = (b4.x & ~snapm) | (S[0] & snapm);
            b4.y = (b4.y & ~snapm) | (S[1] & snapm);
            b4.z = (b4.z & ~snapm) | (S[2] & snapm);
            b4.w = (b4.w & ~snapm) | (S[3] & snapm);
            *reinterpret_cast<GLOBAL_AS u32x4*>(bestw + 4 * g) = b4;
          }
          uint32_t Uq[4][kMscPlanes];
          int d[4];
          group_unsat(st, adjm, U.gbase[g], U.gdeg[g], cnt, S, Uq, d, planes);
          uint32_t F[4] = {0, 0, 0, 0};
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            uint4 x = make_uint4(0, 0, 0, 0);
            if (draw_needed) x = group_block((uint32_t)g, t, rb + i, kTagSweep, k0, k1);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              if (j < cnt) {
                const int k = d[j] - 2 * slice_get(Uq[j], 8 * o + i, planes);
                const bool acc = k <= 0 || accept_pos(k, len, pick(x, j), row);
                F[j] |= (acc ? 1u : 0u) << (8 * o + i);
                dE[i] += acc ? 2 * k : 0;
                nacc[i] += acc ? 1 : 0;
              }
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) F[j] = quad_or(F[j]);
          if (o == 0)
            *reinterpret_cast<uint4*>(st + 4 * g) =
                make_uint4(S[0] ^ F[0], S[1] ^ F[1], S[2] ^ F[2], S[3] ^ F[3]);
        }
      }
      if (c == C - 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int s = quad_lane_sum(dE[i]);
          if ((tid & 63) < 4 && s != 0) atomicAdd(&sh.eacc[t % 3][wl * 32 + 8 * o + i], s);
          dE[i] = 0;
        }
      }
      __syncthreads();
    }
    // end of sweep: the first 32 threads of each word slice own one replica
    if (lt < 32) {
      const int q = wl * 32 + lt;
      const int r = r0 + lt;
      const int e = sh.E[q] + sh.eacc[t % 3][q];
      sh.eacc[(t + 2) % 3][q] = 0;
      sh.E[q] = e;
      const int cut = (W - e) / 2;
      const bool imp = cut > sh.best_cut[q];
      if (imp) {
        sh.best_cut[q] = cut;
        sh.best_sweep[q] = t;
      }
      // lanes 0..31 of the slice's first wave (TPR is a multiple of 64)
      const unsigned long long bal = __ballot(imp);
      if (lt == 0) sh.snap[wl] = (uint32_t)bal;
      if ((J.flags & kJobTrace) && r < J.R) J.trace[(int64_t)t * J.R + r] = e;
    }
    __syncthreads();
  }

  const uint32_t snapm = sh.snap[wl];
  if (live && o == 0) {
    for (int g = gq; g < n_grp; g += QPR) {
      const uint4 s4 = *reinterpret_cast<const uint4*>(st + 4 * g);
      if (snapm) {
        u32x4 b4 = *reinterpret_cast<const GLOBAL_AS u32x4*>(bestw + 4 * g);
        b4.x = (b4.x & ~snapm) | (s4.x & snapm);
        b4.y = (b4.y & ~snapm) | (s4.y & snapm);
        b4.z = (b4.z & ~snapm) | (s4.z & snapm);
        b4.w = (b4.w & ~snapm) | (s4.w & snapm);
        *reinterpret_cast<GLOBAL_AS u32x4*>(bestw + 4 * g) = b4;
      }
      *reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(J.save) + (int64_t)wi * n_pad + 4 * g) = s4;
    }
  }
  // accepted flips per replica: reuse eacc[3] as the accumulator
  __syncthreads();
  if (tid < kMaxWordsPerBlock * 32) sh.eacc[3][tid] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int s = quad_lane_sum(nacc[i]);
    if ((tid & 63) < 4 && s != 0) atomicAdd(&sh.eacc[3][wl * 32 + 8 * o + i], s);
  }
  __syncthreads();
  if (lt < 32) {
    const int q = wl * 32 + lt;
    const int r = r0 + lt;
    if (r < J.R) {
      const unsigned long long prev = fresh ? 0ull : J.accepts[r];
      J.accepts[r] = prev + (unsigned long long)(uint32_t)sh.eacc[3][q];
      J.energy[r] = sh.E[q];
      J.best_cut[r] = sh.best_cut[q];
      J.best_sweep[r] = sh.best_sweep[q];
    }
  }
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK)
k_msc(const JobDev* __restrict__ jobs, const int2* __restrict__ units,
      const int32_t* __restrict__ list_off, int32_t* __restrict__ ctr, int planes) {
  extern __shared__ __align__(16) uint32_t smem_u[];
  __shared__ MscShared sh;
  int tried = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh.unit = next_unit(list_off, ctr, tried);
    __syncthreads();
    const int u = sh.unit;
    if (u < 0) break;
    const int2 un = units[u];
    const JobDev J = jobs[un.x];  // by value: fields stay in registers
    msc_unit<BLOCK>(J, un.y, smem_u, sh, planes);
  }
}

// ================================================================ msc4
// Multispin form of the degree-4 graphs (unit weights, every vertex of
// degree 4: the tori).  A unit is W replicas (W = 8, 16 or 32) of one
// problem.  The state of position p is a W-bit element (bit b = spin of
// replica r0 + b, set = +1), kept in LDS next to its complement in the
// tiled layout of the FIELD kernel's degree-4 forms; an adjacency entry
// names the neighbour's element or its complement, whichever carries the
// edge's sign, so the element read XOR the vertex's own is the bond's
// unsatisfied mask (w s_v s_u = +1).  A lane takes P = 32 / W groups at
// once, their elements side by side in one register (group h in bits
// h W .. h W + W - 1), so each bitwise operation serves 32 (group, replica)
// pairs whatever W is.
//
// Per slot the four unsatisfied masks are counted bit-sliced into u (three
// planes), and k = 4 - 2u.  Moves with u >= 2 (k <= 0) are accepted; u = 1
// (k = 2) and u = 0 (k = 4) compare the replica's draw with the sweep's
// thresholds.  The compares do not depend on the state: each (group,
// replica) draw is compared with both thresholds into one bit of two masks
// per slot, and the flip mask is F = u1 | u2 | (u0 ? A2 : A4) over the real
// slots.  Accounting: a lane counts, bit-sliced, the flips N of a sweep and
// the sum of u over them; a flip changes the energy by 2 k = 8 - 4 u, so the
// sweep's change is 8 N - 4 sum(u F).  At the end of the sweep the counters
// are summed over the wave, still bit-sliced, and each replica's totals are
// read out by one lane.

template <int W>
struct Msc4Types;
template <>
struct Msc4Types<8> {
  typedef uint8_t E;
  typedef uint16_t Pair;
};
template <>
struct Msc4Types<16> {
  typedef uint16_t E;
  typedef uint32_t Pair;
};
template <>
struct Msc4Types<32> {
  typedef uint32_t E;
  typedef unsigned long long Pair;
};

// Planes of a lane's counters: a (group, replica) bit of a lane meets at
// most kMsc4MaxLaneIters groups per sweep (checked on the host), each with
// at most 4 flips and a sum of u of 16.
constexpr int kMsc4NPlanes = 8;   // flips in one sweep
constexpr int kMsc4UPlanes = 10;  // sum of u over them (also the initial sum of u)

struct Msc4Shared {
  int32_t unit;
  int32_t dE[3][32];  // [t % 3]: energy change of sweep t, per replica of the unit
  int32_t dN[3][32];  // [t % 3]: flips of sweep t
  int32_t usum[32];   // fresh start: sum over positions of u
};

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

// A[j] = 2 A[j] + (x_j <= T) for the four words of a block.  The four
// compares go to separate SGPR pairs before the four adds-with-carry read
// them, so that no compare waits on the previous add (one carry register
// would chain all of them).
__device__ __forceinline__ void shift_in4(uint32_t (&A)[4], const uint4& x, uint32_t T) {
  uint64_t m0, m1, m2, m3;
  asm("v_cmp_ge_u32_e64 %0, %4, %5\n\t"
      "v_cmp_ge_u32_e64 %1, %4, %6\n\t"
      "v_cmp_ge_u32_e64 %2, %4, %7\n\t"
      "v_cmp_ge_u32_e64 %3, %4, %8"
      : "=&s"(m0), "=&s"(m1), "=&s"(m2), "=&s"(m3)
      : "s"(T), "v"(x.x), "v"(x.y), "v"(x.z), "v"(x.w));
  asm("v_addc_co_u32_e64 %0, %4, %0, %0, %4\n\t"
      "v_addc_co_u32_e64 %1, %5, %1, %1, %5\n\t"
      "v_addc_co_u32_e64 %2, %6, %2, %2, %6\n\t"
      "v_addc_co_u32_e64 %3, %7, %3, %3, %7"
      : "+v"(A[0]), "+v"(A[1]), "+v"(A[2]), "+v"(A[3]), "+s"(m0), "+s"(m1), "+s"(m2), "+s"(m3));
}

// n = a + b + c + d of four masks, bit-sliced into three planes.
__device__ __forceinline__ void count4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t& n0,
                                       uint32_t& n1, uint32_t& n2) {
  const uint32_t s = xor3(a, b, c), k = maj3(a, b, c);
  n0 = s ^ d;
  const uint32_t k2 = s & d;
  n1 = k ^ k2;
  n2 = k & k2;
}

// X += Y, bit-sliced (NY <= NX planes; a carry out of plane NX - 1 is
// dropped, which the plane bounds exclude).
template <int NX, int NY>
__device__ __forceinline__ void slice_add_n(uint32_t (&X)[NX], const uint32_t (&Y)[NY]) {
  uint32_t c = X[0] & Y[0];
  X[0] ^= Y[0];
#pragma unroll
  for (int p = 1; p < NX; ++p) {
    const uint32_t x = X[p];
    if (p < NY) {
      X[p] = xor3(x, Y[p], c);
      c = maj3(x, Y[p], c);
    } else {
      X[p] = x ^ c;
      c = x & c;
    }
  }
}

// Z holds a lane's counter in its first NP planes (zeros above); it becomes
// the sum over the wave (NP + 6 planes), in every lane.  All lanes take part.
template <int NP, int NZ>
__device__ __forceinline__ void slice_wave_sum(uint32_t (&Z)[NZ]) {
  static_assert(NZ >= NP + 6, "the wave sum needs six more planes");
#pragma unroll
  for (int lvl = 0; lvl < 6; ++lvl) {
    uint32_t c = 0;
#pragma unroll
    for (int p = 0; p < NP + lvl + 1; ++p) {
      const uint32_t y = (uint32_t)__shfl_xor((int)Z[p], 1 << lvl, 64);
      const uint32_t x = Z[p];
      Z[p] = xor3(x, y, c);
      c = maj3(x, y, c);
    }
  }
}

// Value at bit `bit` of a bit-sliced number.
template <int NZ>
__device__ __forceinline__ int slice_value(const uint32_t (&Z)[NZ], int bit) {
  int v = 0;
#pragma unroll
  for (int p = 0; p < NZ; ++p) v |= (int)((Z[p] >> bit) & 1u) << p;
  return v;
}

// LDS byte address base + MUL * (half HI of a packed pair of 16-bit
// entries), one multiply-add.
template <int HI, int MUL>
__device__ __forceinline__ uint32_t lds_entry_addr(uint32_t two, uint32_t base) {
  uint32_t a;
  if (HI)
    asm("v_mad_u32_u16 %0, %1, %3, %2 op_sel:[1,0,0,0]" : "=v"(a) : "v"(two), "v"(base), "n"(MUL));
  else
    asm("v_mad_u32_u16 %0, %1, %3, %2" : "=v"(a) : "v"(two), "v"(base), "n"(MUL));
  return a;
}

template <class T>
__device__ __forceinline__ T lds_load(uint32_t byte_addr) {
  return *(const __attribute__((address_space(3))) T*)(uintptr_t)byte_addr;
}
template <class T>
__device__ __forceinline__ void lds_store(uint32_t byte_addr, T v) {
  *(__attribute__((address_space(3))) T*)(uintptr_t)byte_addr = v;
}

// An element and its complement, as stored.
template <int W>
__device__ __forceinline__ typename Msc4Types<W>::Pair msc4_pair(uint32_t e) {
  typedef typename Msc4Types<W>::Pair Pair;
  if constexpr (W == 32) {
    return (Pair)e | ((Pair)(~e) << 32);
  } else {
    constexpr uint32_t M = (1u << W) - 1u;
    return (Pair)((e & M) | ((~e & M) << W));
  }
}

// Byte offset of replica block r0's element of position p in the [R/32][n_pad]
// word arrays (save, best): the element's word is (r0 / 32, p), its byte
// (r0 mod 32) / 8.
__device__ __forceinline__ int64_t msc4_word_byte(int r0, int n_pad, int p) {
  return ((int64_t)(r0 >> 5) * n_pad + p) * 4 + ((r0 & 31) >> 3);
}

template <int BLOCK, int W>
__device__ void msc4_unit(const JobDev& J, const int block, uint32_t* smem, Msc4Shared& sh) {
  typedef typename Msc4Types<W>::E E;
  typedef typename Msc4Types<W>::Pair Pair;
  constexpr int P = 32 / W;
  constexpr uint32_t WM = W == 32 ? 0xFFFFFFFFu : (1u << (W & 31)) - 1u;
  const int tid = threadIdx.x, lane = tid & 63;
  // a step covers P BLOCK groups of its range in slices of 64: slice
  // h NW + w goes to wave w as its h-th, so lane l of wave w takes groups
  // 64 (h NW + w) + l, h < P.  In a step that ends the range the waves'
  // slices differ by at most one, and slices wholly past the end are
  // skipped by the whole wave.
  constexpr int NW = BLOCK / 64;
  constexpr int HS = 64 * NW;  // group distance between a lane's slices
  const int lane_base = (tid >> 6) * 64 + lane;
  const int r0 = block * W;
  const int live = min(W, J.R - r0);
  const int n_pad = J.n_pad, n_grp = n_pad >> 2;
  const int SW = field_state_words(n_pad);
  const int C = J.n_colours;
  const uint32_t k0 = J.seed_lo, k1 = J.seed_hi;
  const bool fresh = J.t_begin == 0;
  const uint32_t st_base = (uint32_t)(uintptr_t)(lds_i32*)smem;
  uint32_t* rows = smem + ((SW * (int)sizeof(Pair) + 15) & ~15) / 4;
  const GLOBAL_AS u32x4* __restrict__ am = gconst(reinterpret_cast<const u32x4*>(J.adj4m));
  GLOBAL_AS uint8_t* saveb = gmut(reinterpret_cast<uint8_t*>(J.save));
  GLOBAL_AS uint8_t* bestb = gmut(static_cast<uint8_t*>(J.best));
  auto own_addr = [&](int g, int j) { return st_base + (uint32_t)sizeof(Pair) * (uint32_t)tile_word(g, j); };

  for (int i = tid; i < 3 * 32; i += BLOCK) {
    (&sh.dE[0][0])[i] = 0;
    (&sh.dN[0][0])[i] = 0;
  }
  if (tid < 32) sh.usum[tid] = 0;

  // ---- state in: initial draw (tag 1) or given spins, or the saved elements
  for (int g = tid; g < n_grp; g += BLOCK) {
    const int cnt = (J.grp[g] >> kGroupCountShift) + 1;
    uint32_t w4[4] = {0u, 0u, 0u, 0u};
    if (!fresh) {
#pragma unroll
      for (int j = 0; j < 4; ++j) w4[j] = *(const GLOBAL_AS E*)(saveb + msc4_word_byte(r0, n_pad, 4 * g + j));
    } else if (J.flags & kJobInitGiven) {
      for (int b = 0; b < live; ++b)
        for (int j = 0; j < cnt; ++j)
          w4[j] |= (J.init_spins[(int64_t)(r0 + b) * n_pad + 4 * g + j] > 0 ? 1u : 0u) << b;
    } else {
      for (int b = 0; b < W; ++b) {
        const uint4 x = group_block((uint32_t)g, 0, (uint32_t)(r0 + b), kTagInit, k0, k1);
        w4[0] |= (x.x >> 31) << b;
        w4[1] |= (x.y >> 31) << b;
        w4[2] |= (x.z >> 31) << b;
        w4[3] |= (x.w >> 31) << b;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) lds_store<Pair>(own_addr(g, j), msc4_pair<W>(w4[j]));
  }
  const int CH = J.row_chunk;
  stage_row_chunk(J.tqb, J.t_begin, min(CH, J.t_end - J.t_begin), rows, kBondRowWords);
  __syncthreads();

  // Packed state of the lane's groups g_h = gb + HS h (h < P): own
  // elements S[j], unsatisfied masks D[j][e], real slots V[j].  A wave's
  // lanes take 64 consecutive groups per h, so they touch consecutive
  // elements of one tile.  cnt_of(g) is the group's slot count, 0 past the
  // end of its range; such a group reads group gb's data (every access
  // stays valid) and V masks it off.  hn (wave-uniform, >= 1 for a lane
  // with work) counts the wave's slices that reach into the range; the
  // bits of the others stay zero.  All adjacency loads are issued before
  // any element is read.
  uint32_t S[4], V[4], D[4][4];
  auto gather = [&](int gb, int hn, auto cnt_of) {
    u32x4 a[P][2];
    int gs[P];
#pragma unroll
    for (int h = 0; h < P; ++h) {
      if (h == 0 || h < hn) {
        const int cnt = cnt_of(gb + HS * h);
        gs[h] = cnt > 0 ? gb + HS * h : gb;
#pragma unroll
        for (int j = 0; j < 4; ++j) V[j] = (h == 0 ? 0u : V[j]) | ((j < cnt ? WM : 0u) << (h * W));
        a[h][0] = am[2 * gs[h]];
        a[h][1] = am[2 * gs[h] + 1];
      }
    }
#pragma unroll
    for (int h = 0; h < P; ++h) {
      if (h > 0 && h >= hn) break;
      // one group's reads at a time, so that few loaded elements are live
      __builtin_amdgcn_sched_barrier(0);
      const uint32_t ent[8] = {a[h][0].x, a[h][0].y, a[h][0].z, a[h][0].w,
                               a[h][1].x, a[h][1].y, a[h][1].z, a[h][1].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t s = lds_load<E>(own_addr(gs[h], j));
        const uint32_t n0 = lds_load<E>(lds_entry_addr<0, sizeof(E)>(ent[2 * j], st_base));
        const uint32_t n1 = lds_load<E>(lds_entry_addr<1, sizeof(E)>(ent[2 * j], st_base));
        const uint32_t n2 = lds_load<E>(lds_entry_addr<0, sizeof(E)>(ent[2 * j + 1], st_base));
        const uint32_t n3 = lds_load<E>(lds_entry_addr<1, sizeof(E)>(ent[2 * j + 1], st_base));
        if (h == 0) {
          S[j] = s;
          D[j][0] = n0;
          D[j][1] = n1;
          D[j][2] = n2;
          D[j][3] = n3;
        } else {
          S[j] |= s << (h * W);
          D[j][0] |= n0 << (h * W);
          D[j][1] |= n1 << (h * W);
          D[j][2] |= n2 << (h * W);
          D[j][3] |= n3 << (h * W);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) D[j][e] ^= S[j];
  };

  // slices of the wave at step base gb (lane 0's group) that start before
  // the end g1 of the range, at most P
  auto slices_in = [&](int gb_lane0, int g1) {
    const int left = g1 - gb_lane0;
    return left <= 0 ? 0 : min(P, (left + HS - 1) / HS);
  };

  // ---- initial energy: E = sum_p u_p - M (each unsatisfied bond counted at
  // both ends is 2 U, and E = 2 U - M)
  int E_r = 0, best_cut_r = 0, best_sweep_r = 0;
  unsigned long long acc_r = 0;
  uint32_t snapW = 0;
  if (fresh) {
    uint32_t AU[kMsc4UPlanes + 6];  // the top six planes take the wave sum's carries
#pragma unroll
    for (int p = 0; p < kMsc4UPlanes + 6; ++p) AU[p] = 0u;
    for (int gb = lane_base; gb < n_grp; gb += P * BLOCK) {
      const int hn = slices_in(__builtin_amdgcn_readfirstlane(gb - lane), n_grp);
      gather(gb, hn, [&](int g) { return g < n_grp ? (J.grp[g] >> kGroupCountShift) + 1 : 0; });
      uint32_t u[4][3];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        count4(D[j][0], D[j][1], D[j][2], D[j][3], u[j][0], u[j][1], u[j][2]);
#pragma unroll
        for (int q = 0; q < 3; ++q) u[j][q] &= V[j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) slice_add_n(AU, u[j]);
    }
    slice_wave_sum<kMsc4UPlanes>(AU);
    if (lane < 32) {
      const int v = slice_value(AU, lane);
      if (v) atomicAdd(&sh.usum[lane & (W - 1)], v);
    }
    __syncthreads();
    if (lane < W) {
      E_r = sh.usum[lane] - J.M;
      best_cut_r = (J.W - E_r) / 2;
      best_sweep_r = -1;
    }
    snapW = WM;  // the initial state is written during sweep 0
  } else if (lane < live) {
    E_r = J.energy[r0 + lane];
    best_cut_r = J.best_cut[r0 + lane];
    best_sweep_r = J.best_sweep[r0 + lane];
    acc_r = J.accepts[r0 + lane];
  }

  int tc = 0;
  for (int t = J.t_begin; t < J.t_end; ++t) {
    if (tc == CH) {
      stage_row_chunk(J.tqb, t, min(CH, J.t_end - t), rows, kBondRowWords);
      tc = 0;
      __syncthreads();
    }
    const uint32_t* row = rows + tc * kBondRowWords;
    ++tc;
    const uint32_t T2 = __builtin_amdgcn_readfirstlane(row[4]);
    const uint32_t T4 = __builtin_amdgcn_readfirstlane(row[5]);
    const int bound = __builtin_amdgcn_readfirstlane((int)row[7]);
    const bool need2 = bound >= 4, need4 = bound >= 5;
    const uint32_t snap32 = snapW * (W == 8 ? 0x01010101u : W == 16 ? 0x00010001u : 1u);
    uint32_t AN[kMsc4NPlanes], AU[kMsc4UPlanes];
#pragma unroll
    for (int p = 0; p < kMsc4NPlanes; ++p) AN[p] = 0u;
#pragma unroll
    for (int p = 0; p < kMsc4UPlanes; ++p) AU[p] = 0u;
    bool worked = false;
    for (int c = 0; c < C; ++c) {
      const int g0 = J.cls[2 * c], g1 = J.cls[2 * c + 1];
      const int cnt_last = g1 > g0 ? (J.grp[g1 - 1] >> kGroupCountShift) + 1 : 0;
      for (int gb = g0 + lane_base; gb < g1; gb += P * BLOCK) {
        worked = true;
        const int hn = slices_in(__builtin_amdgcn_readfirstlane(gb - lane), g1);
        // draws of the lane's groups, compared with both thresholds; they do
        // not depend on the state, so they come first, four independent
        // blocks at a time (bits are shifted in from the highest: group
        // P-1, replica W-1 first)
        uint32_t A2[4] = {0u, 0u, 0u, 0u}, A4[4] = {0u, 0u, 0u, 0u};
        if (need4) {
#pragma unroll
          for (int h = P - 1; h >= 0; --h) {
            if (h >= hn) continue;
            const uint32_t g = (uint32_t)(gb + HS * h);
            for (int b = W - 1; b >= 0; b -= 4) {
              uint4 x[4];
              const uint32_t rs[4] = {(uint32_t)(r0 + b), (uint32_t)(r0 + b - 1), (uint32_t)(r0 + b - 2),
                                      (uint32_t)(r0 + b - 3)};
              philox10_x4(t, g, rs, kTagSweep, k0, k1, x);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                shift_in4(A2, x[i], T2);
                shift_in4(A4, x[i], T4);
              }
              // four blocks in flight, not more (registers)
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        } else if (need2) {
#pragma unroll
          for (int h = P - 1; h >= 0; --h) {
            if (h >= hn) continue;
            const uint32_t g = (uint32_t)(gb + HS * h);
            for (int b = W - 1; b >= 0; b -= 4) {
              uint4 x[4];
              const uint32_t rs[4] = {(uint32_t)(r0 + b), (uint32_t)(r0 + b - 1), (uint32_t)(r0 + b - 2),
                                      (uint32_t)(r0 + b - 3)};
              philox10_x4(t, g, rs, kTagSweep, k0, k1, x);
#pragma unroll
              for (int i = 0; i < 4; ++i) shift_in4(A2, x[i], T2);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
        gather(gb, hn, [&](int g) { return g >= g1 ? 0 : g == g1 - 1 ? cnt_last : 4; });
        // lazy best-state snapshot: these groups' end-of-last-sweep spins
        if (snap32) {
          // (rare after the first sweeps: a rolled loop, so that it adds
          // no registers to the unrolled visit)
#pragma unroll 1
          for (int h = 0; h < P; ++h) {
            const int g = gb + HS * h;
            if (g < g1) {
              GLOBAL_AS E* bp = (GLOBAL_AS E*)(bestb + msc4_word_byte(r0, n_pad, 4 * g));
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                if ((V[j] >> (h * W)) & 1u) {
                  // element j of the group is 4 bytes further per slot
                  GLOBAL_AS E* q = (GLOBAL_AS E*)((GLOBAL_AS uint8_t*)bp + 4 * j);
                  const uint32_t old = *q, sv = (S[j] >> (h * W)) & WM;
                  *q = (E)((old & ~snapW) | (sv & snapW));
                }
              }
            }
          }
        }
        // flips, counts and the new state
        uint32_t F[4], uF[4][3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          uint32_t u0, u1, u2;
          count4(D[j][0], D[j][1], D[j][2], D[j][3], u0, u1, u2);
          const uint32_t sel = (u0 & A2[j]) | (~u0 & A4[j]);
          F[j] = (u1 | u2 | sel) & V[j];
          uF[j][0] = u0 & F[j];
          uF[j][1] = u1 & F[j];
          uF[j][2] = u2 & F[j];
        }
        uint32_t nf[3];
        count4(F[0], F[1], F[2], F[3], nf[0], nf[1], nf[2]);
        // sum of u over the flips: (uF0 + uF1) + (uF2 + uF3), 5 planes
        uint32_t s01[4], s23[4], su[5];
        {
          uint32_t cy = uF[0][0] & uF[1][0];
          s01[0] = uF[0][0] ^ uF[1][0];
          s01[1] = xor3(uF[0][1], uF[1][1], cy);
          cy = maj3(uF[0][1], uF[1][1], cy);
          s01[2] = xor3(uF[0][2], uF[1][2], cy);
          s01[3] = maj3(uF[0][2], uF[1][2], cy);
          cy = uF[2][0] & uF[3][0];
          s23[0] = uF[2][0] ^ uF[3][0];
          s23[1] = xor3(uF[2][1], uF[3][1], cy);
          cy = maj3(uF[2][1], uF[3][1], cy);
          s23[2] = xor3(uF[2][2], uF[3][2], cy);
          s23[3] = maj3(uF[2][2], uF[3][2], cy);
          cy = s01[0] & s23[0];
          su[0] = s01[0] ^ s23[0];
#pragma unroll
          for (int q = 1; q < 4; ++q) {
            su[q] = xor3(s01[q], s23[q], cy);
            cy = maj3(s01[q], s23[q], cy);
          }
          su[4] = cy;
        }
        slice_add_n(AN, nf);
        slice_add_n(AU, su);
#pragma unroll
        for (int h = 0; h < P; ++h) {
          __builtin_amdgcn_sched_barrier(0);
          const int g = gb + HS * h;
          if (g < g1) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const uint32_t e = (S[j] ^ F[j]) >> (h * W);
              lds_store<Pair>(own_addr(g, j), msc4_pair<W>(e));
            }
          }
        }
      }
      if (c == C - 1) {
        // the sweep's totals, summed over the wave bit-sliced; lane q < 32
        // reads bit q, which belongs to replica q mod W
        if (__builtin_amdgcn_ballot_w64(worked) != 0) {
          uint32_t ZN[kMsc4NPlanes + 6], ZU[kMsc4UPlanes + 6];
#pragma unroll
          for (int p = 0; p < kMsc4NPlanes + 6; ++p) ZN[p] = p < kMsc4NPlanes ? AN[p] : 0u;
#pragma unroll
          for (int p = 0; p < kMsc4UPlanes + 6; ++p) ZU[p] = p < kMsc4UPlanes ? AU[p] : 0u;
          slice_wave_sum<kMsc4NPlanes>(ZN);
          slice_wave_sum<kMsc4UPlanes>(ZU);
          if (lane < 32) {
            const int n = slice_value(ZN, lane), us = slice_value(ZU, lane);
            if (n != 0) {
              atomicAdd(&sh.dN[t % 3][lane & (W - 1)], n);
              atomicAdd(&sh.dE[t % 3][lane & (W - 1)], 8 * n - 4 * us);
            }
          }
        }
      }
      __syncthreads();
    }
    // end of sweep t: every wave keeps the unit's per-replica scalars in its
    // lanes 0 .. W-1
    bool imp = false;
    if (lane < W) {
      E_r += sh.dE[t % 3][lane];
      acc_r += (unsigned long long)sh.dN[t % 3][lane];
      const int cut = (J.W - E_r) / 2;
      imp = lane < live && cut > best_cut_r;
      if (imp) {
        best_cut_r = cut;
        best_sweep_r = t;
      }
    }
    snapW = (uint32_t)__builtin_amdgcn_ballot_w64(imp) & WM;
    if (tid < W) {
      sh.dE[(t + 2) % 3][tid] = 0;
      sh.dN[(t + 2) % 3][tid] = 0;
    }
    if ((J.flags & kJobTrace) && tid < live) J.trace[(int64_t)t * J.R + r0 + tid] = E_r;
  }

  // ---- state out, and the snapshot of the last sweep when it improved
  for (int g = tid; g < n_grp; g += BLOCK) {
    const int cnt = (J.grp[g] >> kGroupCountShift) + 1;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t e = lds_load<E>(own_addr(g, j));
      const int64_t o = msc4_word_byte(r0, n_pad, 4 * g + j);
      if (snapW && j < cnt) {
        GLOBAL_AS E* bp = (GLOBAL_AS E*)(bestb + o);
        *bp = (E)(((uint32_t)*bp & ~snapW) | (e & snapW));
      }
      if (J.save) *(GLOBAL_AS E*)(saveb + o) = (E)e;
    }
  }
  if (tid < live) {
    J.accepts[r0 + tid] = acc_r;
    J.energy[r0 + tid] = E_r;
    J.best_cut[r0 + tid] = best_cut_r;
    J.best_sweep[r0 + tid] = best_sweep_r;
  }
}

template <int BLOCK, int W>
__global__ void __launch_bounds__(BLOCK)
k_msc4(const JobDev* __restrict__ jobs, const int2* __restrict__ units,
       const int32_t* __restrict__ list_off, int32_t* __restrict__ ctr) {
  extern __shared__ __align__(16) uint32_t smem_m4[];
  __shared__ Msc4Shared sh;
  int tried = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh.unit = next_unit(list_off, ctr, tried);
    __syncthreads();
    const int u = sh.unit;
    if (u < 0) break;
    const int2 un = units[u];
    const JobDev J = jobs[un.x];  // by value: fields stay in registers
    msc4_unit<BLOCK, W>(J, un.y, smem_m4, sh);
  }
}

// ================================================================ utils
// Argmax over replicas of each job: key = (best_cut + 2^31 mod 2^32) << 32
// | ~r, so the largest key is the largest cut with the lowest replica index
// (the offset is a sign-bit flip in unsigned arithmetic).
__global__ void k_argmax(const JobDev* jobs) {
  const JobDev& J = jobs[blockIdx.x];
  unsigned long long key = 0;
  for (int r = threadIdx.x; r < J.R; r += blockDim.x) {
    const unsigned long long k =
        ((unsigned long long)((uint32_t)J.best_cut[r] ^ 0x80000000u) << 32) |
        (unsigned long long)(0xFFFFFFFFu - (uint32_t)r);
    key = k > key ? k : key;
  }
  key = wave_max_u64(key);
  __shared__ unsigned long long part[16];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = part[i] > m ? part[i] : m;
    *J.argmax = m;
  }
}

__global__ void k_gather(const void* buf, int layout, int R, int n_pad, int r,
                         const int32_t* pos, int n, int32_t* out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int p = pos[v];
  int val = 0;
  switch (layout) {
    case kLayoutNR_I8: val = static_cast<const int8_t*>(buf)[(int64_t)p * R + r]; break;
    case kLayoutRN_I8: val = static_cast<const int8_t*>(buf)[(int64_t)r * n_pad + p]; break;
    case kLayoutRN_Spin:
      val = (static_cast<const int32_t*>(buf)[(int64_t)r * n_pad + p] & 1) ? 1 : -1;
      break;
    case kLayoutRN_Field: val = static_cast<const int32_t*>(buf)[(int64_t)r * n_pad + p] >> 1; break;
    case kLayoutNR_I32: val = static_cast<const int32_t*>(buf)[(int64_t)p * R + r]; break;
    case kLayoutWords:
      val = ((static_cast<const uint32_t*>(buf)[(int64_t)(r >> 5) * n_pad + p] >> (r & 31)) & 1u) ? 1 : -1;
      break;
  }
  out[v] = val;
}

// Every replica's int8 state [R][n_pad] (position order) into [R][n]
// (original order): one lane per (replica, vertex).
__global__ void k_gather_states(const int8_t* src, int R, int n_pad, const int32_t* pos, int n,
                                int8_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)R * n) return;
  const int r = (int)(i / n), v = (int)(i - (int64_t)r * n);
  out[i] = src[(int64_t)r * n_pad + pos[v]];
}

__global__ void k_fill_i32(int32_t* p, int32_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// ================================================================ tempering
// Start of a tempering run: replica set K + k at temperature k, no
// exchanges yet.
__global__ void k_pt_init(SwapDev X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int R = X.K * X.n_sets;
  if (i < R) {
    X.temp[i] = i % X.K;
    X.slot[i] = i;
  }
  if (i < X.n_sets * (X.K - 1)) X.swaps[i] = 0;
}

// Exchange round m: pairs (k, k+1) with k of m's parity, one lane per pair
// and set (the pairs of a round are disjoint).  The replicas a (at k) and b
// (at k+1) exchange temperatures with the Metropolis probability of the
// product of Boltzmann weights, min(1, exp(-(beta_k+1 - beta_k)(E_a - E_b))):
// always when q = (E_a - E_b) / 2 <= 0 (energies of one problem differ by an
// even number), else when the round's draw is below the quantised
// threshold of q.
// (Also zeroes clear8[0..7] when given: the persistent launch's list
// cursors, for the next segment.)
// Houdayer cluster move of pair p at temperature k in round m (after sweep
// t): the replicas a (set 2p) and b (set 2p+1) at k disagree on the sites
// D; the seed is the (u mod |D|)-th site of D in ascending original id, u
// word 0 of Philox(m, k, p, 4); its connected component in the subgraph
// induced by D flips in both replicas (which keeps E_a + E_b), and both
// replicas' fields and energies are recomputed.  One workgroup per (p, k).
// The two replicas' spins, D and the cluster marks are bitmasks over the
// positions in LDS; the component is found by union-find (a search from
// the seed would take one dependent step per level of the cluster, and
// clusters of thousands of sites have hundreds).  With X.stage the parents
// and the position CSR are staged in LDS too, else the parents live in the
// workgroup's global scratch.
constexpr int kClusterThreads = 1024;

__global__ void __launch_bounds__(kClusterThreads) k_houdayer(ClusterDev X, int m, int t) {
  extern __shared__ uint32_t lds[];
  __shared__ int scan[kClusterThreads / 64];
  __shared__ int sh_i0, sh_tail;
  __shared__ int esum[2];
  const int n_pad = X.n_pad, n = X.n;
  const int W = (n_pad + 31) / 32;
  uint32_t* dmask = lds;
  uint32_t* abits = lds + W;
  uint32_t* bbits = lds + 2 * W;
  uint32_t* mk = lds + 3 * W;
  const int nk = X.K - X.from;
  const int p = blockIdx.x / nk, k = X.from + (int)(blockIdx.x - p * nk);
  const int tid = threadIdx.x;
  const int a = X.slot[(2 * p) * X.K + k], b = X.slot[(2 * p + 1) * X.K + k];
  const bool plain = X.packed == nullptr;
  const int n_adj = X.row[n_pad];
  // union-find parents of the positions (LDS when staged, else the
  // workgroup's global scratch); staged: 16-bit row offsets, neighbour
  // positions and vertex positions in LDS
  const bool stage = X.stage != 0;
  int32_t* parent = stage ? reinterpret_cast<int32_t*>(lds + 4 * W) : X.queue + (int64_t)blockIdx.x * n_pad;
  uint16_t* row16 = reinterpret_cast<uint16_t*>(lds + 4 * W + n_pad);
  uint16_t* adj16 = row16 + n_pad + 1;
  uint16_t* pos16 = adj16 + n_adj;
  // unit weights on fewer than 2^15 positions: an entry also carries the
  // sign of its weight in bit 15
  const bool signs = stage && X.unit;
  if (stage) {
    copy_in(row16, X.row, n_pad + 1, [](int32_t x) { return (uint16_t)x; });
    copy_in(pos16, X.pos, n, [](int32_t x) { return (uint16_t)x; });
    if (signs) {
      // two passes keep each copy a plain map of one source array
      copy_in(adj16, X.adj, n_adj, [](int32_t x) { return (uint16_t)x; });
      __syncthreads();
      for (int i0 = tid; i0 < n_adj; i0 += 8 * kClusterThreads) {
        int32_t wv[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) wv[z] = X.wgt[min(i0 + z * kClusterThreads, n_adj - 1)];
#pragma unroll
        for (int z = 0; z < 8; ++z)
          if (i0 + z * kClusterThreads < n_adj && wv[z] > 0) adj16[i0 + z * kClusterThreads] |= 0x8000u;
      }
    } else {
      copy_in(adj16, X.adj, n_adj, [](int32_t x) { return (uint16_t)x; });
    }
  }
  auto row_at = [&](int i) -> int { return stage ? (int)row16[i] : X.row[i]; };
  auto adj_at = [&](int e) -> int { return stage ? (int)(adj16[e] & 0x7FFFu) : X.adj[e]; };
  auto pos_at = [&](int v) -> int { return stage ? (int)pos16[v] : X.pos[v]; };

  auto state_bit = [&](int r, int q) -> uint32_t {
    return plain ? (X.spins[(int64_t)q * X.R + r] > 0 ? 1u : 0u) : (uint32_t)(X.packed[(int64_t)r * n_pad + q] & 1);
  };
  auto real = [&](int q) { return (q & 3) <= (X.grp[q >> 2] >> kGroupCountShift); };
  // pending lazy snapshots of the plain path: the last sweep improved, so
  // its end state is the best state; take it before the move changes it
  const bool snap_a = plain && X.snap[a] == t, snap_b = plain && X.snap[b] == t;
  if (snap_a || snap_b) {
    for (int q = tid; q < n_pad; q += kClusterThreads) {
      if (snap_a) X.best[(int64_t)q * X.R + a] = X.spins[(int64_t)q * X.R + a];
      if (snap_b) X.best[(int64_t)q * X.R + b] = X.spins[(int64_t)q * X.R + b];
    }
  }
  // bitmasks: a wave reads 64 consecutive positions and ballots them into
  // two words
  const int lane = tid & 63;
  for (int q0 = tid - lane; q0 < n_pad; q0 += kClusterThreads) {
    const int q = q0 + lane;
    const bool in = q < n_pad;
    const uint64_t ba = __ballot(in && state_bit(a, q));
    const uint64_t bb = __ballot(in && state_bit(b, q));
    const uint64_t br = __ballot(in && real(q));
    if (lane < 2 && (q0 >> 5) + lane < W) {
      const int i = (q0 >> 5) + lane;
      const uint32_t wa = (uint32_t)(ba >> (32 * lane)), wb = (uint32_t)(bb >> (32 * lane));
      abits[i] = wa;
      bbits[i] = wb;
      dmask[i] = (wa ^ wb) & (uint32_t)(br >> (32 * lane));
      mk[i] = 0u;
    }
  }
  for (int q = tid; q < n_pad; q += kClusterThreads) parent[q] = q;
  if (tid == 0) sh_tail = 0;
  __syncthreads();
  if (tid == 0) {
    if (snap_a) X.snap[a] = -2;
    if (snap_b) X.snap[b] = -2;
  }
  auto in_d = [&](int q) { return (dmask[q >> 5] >> (q & 31)) & 1u; };
  // |D| and the seed: ids in contiguous chunks per lane, an exclusive scan
  const int chunk = (n + kClusterThreads - 1) / kClusterThreads;
  const int v0 = min(n, tid * chunk), v1 = min(n, v0 + chunk);
  int cnt = 0;
  for (int v = v0; v < v1; ++v) cnt += (int)in_d(pos_at(v));
  // exclusive scan of the counts: within each wave by lane shuffles, then
  // over the waves' totals
  int incl = cnt;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) scan[tid >> 6] = incl;
  if (tid == 0) sh_i0 = -1;
  __syncthreads();
  int before = 0, total = 0;
  for (int wv = 0; wv < kClusterThreads / 64; ++wv) {
    const int c = scan[wv];
    before += wv < (tid >> 6) ? c : 0;
    total += c;
  }
  const int excl = before + incl - cnt;
  if (total == 0) return;  // uniform: the replicas agree everywhere
  const uint4 x = philox10((uint32_t)m, (uint32_t)k, (uint32_t)p, kTagCluster, X.seed_lo, X.seed_hi);
  const int j = (int)(x.x % (uint32_t)total);
  if (j >= excl && j < excl + cnt) {
    int left = j - excl;
    for (int v = v0; v < v1; ++v)
      if (in_d(pos_at(v)) && left-- == 0) {
        sh_i0 = pos_at(v);
        break;
      }
  }
  __syncthreads();
  if (sh_i0 < 0) return;  // (uniform; cannot happen: j < |D|)
  // Connected components of the subgraph induced by D by concurrent
  // union-find: every edge inside D hooks the larger of its ends' roots
  // onto the smaller with a compare-and-swap (retrying when another lane
  // moved the root first), and finds halve their paths.  The components,
  // and so the seed's cluster, do not depend on the order of the hooks.
  volatile int32_t* par = parent;
  auto find = [&](int v) {
    int p = par[v];
    while (p != v) {
      const int g = par[p];
      if (g != p) par[v] = g;
      v = p;
      p = g;
    }
    return v;
  };
  for (int q = tid; q < n_pad; q += kClusterThreads) {
    if (!in_d(q)) continue;
    const int e1 = row_at(q + 1);
    for (int e = row_at(q); e < e1; ++e) {
      const int u = adj_at(e);
      if (u <= q || !in_d(u)) continue;
      int x = q, y = u;
      for (;;) {
        x = find(x);
        y = find(y);
        if (x == y) break;
        if (x > y) {
          const int z = x;
          x = y;
          y = z;
        }
        if (atomicCAS(&parent[y], y, x) == y) break;
      }
    }
  }
  __syncthreads();
  // the seed's cluster as marks, and its size
  const int root = find(sh_i0);
  int mine = 0;
  const int lane2 = tid & 63;
  for (int q0 = tid - lane2; q0 < n_pad; q0 += kClusterThreads) {
    const int q = q0 + lane2;
    const bool inc = q < n_pad && in_d(q) && find(q) == root;
    const uint64_t bm = __ballot(inc);
    if (lane2 < 2 && (q0 >> 5) + lane2 < W) mk[(q0 >> 5) + lane2] = (uint32_t)(bm >> (32 * lane2));
    mine += inc ? 1 : 0;
  }
  {
    const int s2 = wave_sum(mine);
    if (lane2 == 0 && s2 != 0) atomicAdd(&sh_tail, s2);
  }
  __syncthreads();
  const int size = sh_tail;
  // flip the cluster in both replicas (the marks are exactly the cluster)
  for (int i = tid; i < W; i += kClusterThreads) {
    abits[i] ^= mk[i];
    bbits[i] ^= mk[i];
  }
  if (tid < 2) esum[tid] = 0;
  __syncthreads();
  // fields and energies from scratch: h = -sum w s, E = -1/2 sum s h
  auto bit_l = [&](const uint32_t* bits, int q) -> int { return (int)((bits[q >> 5] >> (q & 31)) & 1u); };
  int part[2] = {0, 0};
  for (int q = tid; q < n_pad; q += kClusterThreads) {
    if (!real(q)) continue;
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      const uint32_t* bits = z ? bbits : abits;
      const int r = z ? b : a;
      int h = 0;
      const int e1 = row_at(q + 1);
      if (signs) {
        // w = +1 (bit 15 set) or -1: h = -sum w s
        for (int e = row_at(q); e < e1; ++e) {
          const int en = adj16[e];
          h += ((en >> 15) ^ bit_l(bits, en & 0x7FFF)) ? 1 : -1;
        }
      } else {
        for (int e = row_at(q); e < e1; ++e) h -= X.wgt[e] * (bit_l(bits, adj_at(e)) ? 1 : -1);
      }
      const int sb = bit_l(bits, q);
      part[z] += sb ? h : -h;
      if (plain) {
        X.spins[(int64_t)q * X.R + r] = (int8_t)(sb ? 1 : -1);
        X.field[(int64_t)q * X.R + r] = h;
      } else {
        X.packed[(int64_t)r * n_pad + q] = (h << 1) | sb;
      }
    }
  }
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    const int s = wave_sum(part[z]);
    if ((tid & 63) == 0 && s != 0) atomicAdd(&esum[z], s);
  }
  __syncthreads();
  if (tid == 0) {
    X.energy[a] = -esum[0] / 2;
    X.energy[b] = -esum[1] / 2;
    X.moves[p * X.K + k] += 1;
    X.sites[p * X.K + k] += size;
  }
}

__global__ void k_swap(SwapDev X, int m, int32_t* clear8) {
  const int per_set = (X.K - (m & 1)) / 2;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (clear8 && i < 8) clear8[i] = 0;
  if (per_set <= 0 || i >= X.n_sets * per_set) return;
  const int set = i / per_set;
  const int k = (m & 1) + 2 * (i - set * per_set);
  int32_t* sl = X.slot + set * X.K;
  const int a = sl[k], b = sl[k + 1];
  const int q = (X.energy[a] - X.energy[b]) / 2;
  bool accept = q <= 0;
  if (!accept) {
    const int len = X.len[k];
    const uint4 x = philox10((uint32_t)m, (uint32_t)k, (uint32_t)set, kTagSwap, X.seed_lo, X.seed_hi);
    accept = len < 0 || (q <= len && x.x <= X.tq[X.off[k] + q - 1]);
  }
  if (accept) {
    sl[k] = b;
    sl[k + 1] = a;
    X.temp[a] = k + 1;
    X.temp[b] = k;
    ++X.swaps[set * (X.K - 1) + k];
  }
}

template <int BLOCK>
hipError_t launch_field_t(const LaunchPersistent& L, hipStream_t s) {
  switch (L.adj) {
    case kAdjHbm:
      hipLaunchKernelGGL((k_field<BLOCK, kAdjHbm>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s,
                         L.jobs, L.units, L.list_off, L.ctr);
      break;
    case kAdjLds:
      hipLaunchKernelGGL((k_field<BLOCK, kAdjLds>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s,
                         L.jobs, L.units, L.list_off, L.ctr);
      break;
    case kAdjLdsDeg4:
      hipLaunchKernelGGL((k_field<BLOCK, kAdjLdsDeg4>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s,
                         L.jobs, L.units, L.list_off, L.ctr);
      break;
    case kAdjPerJob:
      hipLaunchKernelGGL((k_field<BLOCK, kAdjPerJob>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s,
                         L.jobs, L.units, L.list_off, L.ctr);
      break;
    case kAdjHbmDeg4:
      hipLaunchKernelGGL((k_field<BLOCK, kAdjHbmDeg4>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s,
                         L.jobs, L.units, L.list_off, L.ctr);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int BLOCK>
const void* field_kernel(int adj) {
  return adj == kAdjLds       ? (const void*)k_field<BLOCK, kAdjLds>
         : adj == kAdjLdsDeg4 ? (const void*)k_field<BLOCK, kAdjLdsDeg4>
         : adj == kAdjPerJob  ? (const void*)k_field<BLOCK, kAdjPerJob>
         : adj == kAdjHbmDeg4 ? (const void*)k_field<BLOCK, kAdjHbmDeg4>
                              : (const void*)k_field<BLOCK, kAdjHbm>;
}

template <int BLOCK>
hipError_t launch_msc_t(const LaunchPersistent& L, hipStream_t s) {
  switch (L.width) {
    case 0:
      hipLaunchKernelGGL(k_msc<BLOCK>, dim3(L.grid), dim3(BLOCK), L.lds_bytes, s, L.jobs,
                         L.units, L.list_off, L.ctr, L.planes);
      break;
    case 8:
      hipLaunchKernelGGL((k_msc4<BLOCK, 8>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s, L.jobs,
                         L.units, L.list_off, L.ctr);
      break;
    case 16:
      hipLaunchKernelGGL((k_msc4<BLOCK, 16>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s, L.jobs,
                         L.units, L.list_off, L.ctr);
      break;
    case 32:
      hipLaunchKernelGGL((k_msc4<BLOCK, 32>), dim3(L.grid), dim3(BLOCK), L.lds_bytes, s, L.jobs,
                         L.units, L.list_off, L.ctr);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The multispin kernel of a width (0 = the general form).
template <int BLOCK>
const void* msc_kernel(int width) {
  return width == 8    ? (const void*)k_msc4<BLOCK, 8>
         : width == 16 ? (const void*)k_msc4<BLOCK, 16>
         : width == 32 ? (const void*)k_msc4<BLOCK, 32>
                       : (const void*)k_msc<BLOCK>;
}

template <typename K>
int occupancy_of(K kernel, int block, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, lds) != hipSuccess) return 0;
  return n;
}

inline int blocks_for(int64_t n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// ================================================================ launchers
hipError_t launch_plain_anneal(const PlainDev& P, const PlainPlan& plan, hipStream_t s) {
  const int B = 256;
  const int n_grp = P.n_pad >> 2;
  const int t_end = plan.t_end < 0 ? plan.S : plan.t_end;
  if (plan.t_begin == 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(P.R, B)), dim3(B), 0, s, P.eacc, 0, (int64_t)P.R);
    hipLaunchKernelGGL(k_plain_init, dim3(blocks_for((int64_t)n_grp * P.R, B)), dim3(B), 0, s, P);
    hipLaunchKernelGGL(k_plain_fields, dim3(blocks_for((int64_t)P.n_pad * P.R, B)), dim3(B), 0, s, P);
    hipLaunchKernelGGL(k_plain_init_best, dim3(blocks_for(P.R, B)), dim3(B), 0, s, P);
  }
  for (int t = plan.t_begin; t < t_end; ++t) {
    for (int c = 0; c < plan.C; ++c) {
      const int g0 = plan.cls[2 * c], g1 = plan.cls[2 * c + 1];
      if (g1 > g0)
        hipLaunchKernelGGL(k_plain_sweep, dim3(blocks_for((int64_t)(g1 - g0) * P.R, B)), dim3(B), 0,
                           s, P, t, g0, g1);
    }
    hipLaunchKernelGGL(k_plain_eos, dim3(blocks_for(P.R, B)), dim3(B), 0, s, P, t, plan.S);
    if (plan.swap && (t + 1) % plan.swap_every == 0) {
      const int m = (t + 1) / plan.swap_every - 1;
      hipError_t e = plan.cluster ? launch_houdayer(*plan.cluster, m, t, s) : hipSuccess;
      if (e != hipSuccess) return e;
      e = launch_swap(*plan.swap, m, nullptr, s);
      if (e != hipSuccess) return e;
    }
  }
  // a pending lazy snapshot of the last sweep (a later range's first sweep
  // would take the same spins again)
  hipLaunchKernelGGL(k_plain_flush, dim3(blocks_for((int64_t)P.n_pad * P.R, B)), dim3(B), 0, s, P,
                     t_end - 1);
  return hipGetLastError();
}

hipError_t launch_field(const LaunchPersistent& L, int block, hipStream_t s) {
  switch (block) {
    case 256: return launch_field_t<256>(L, s);
    case 512: return launch_field_t<512>(L, s);
    case 1024: return launch_field_t<1024>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_msc(const LaunchPersistent& L, int block, hipStream_t s) {
  switch (block) {
    case 256: return launch_msc_t<256>(L, s);
    case 512: return launch_msc_t<512>(L, s);
    case 1024:
      // the general form runs 256 or 512 threads
      if (L.width == 0) return hipErrorInvalidValue;
      return launch_msc_t<1024>(L, s);
    default: return hipErrorInvalidValue;
  }
}

int persistent_occupancy(int path, int block, int adj, size_t lds_bytes) {
  if (path == 2) {
    switch (block) {
      case 256: return occupancy_of(field_kernel<256>(adj), 256, lds_bytes);
      case 512: return occupancy_of(field_kernel<512>(adj), 512, lds_bytes);
      case 1024: return occupancy_of(field_kernel<1024>(adj), 1024, lds_bytes);
    }
  } else {
    // adj: the multispin width (0 = the general form)
    switch (block) {
      case 256: return occupancy_of(msc_kernel<256>(adj), 256, lds_bytes);
      case 512: return occupancy_of(msc_kernel<512>(adj), 512, lds_bytes);
      case 1024: return adj ? occupancy_of(msc_kernel<1024>(adj), 1024, lds_bytes) : 0;
    }
  }
  return 0;
}

hipError_t set_persistent_lds_limit(int path, int block, size_t lds_bytes) {
  const void* f = nullptr;
  if (path == 2) {
    for (int adj : {kAdjLds, kAdjLdsDeg4, kAdjPerJob, kAdjHbmDeg4}) {
      const void* k = block == 256 ? field_kernel<256>(adj)
                                   : block == 512 ? field_kernel<512>(adj) : field_kernel<1024>(adj);
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
      if (e != hipSuccess) return e;
    }
    f = block == 256 ? field_kernel<256>(kAdjHbm)
                     : block == 512 ? field_kernel<512>(kAdjHbm) : field_kernel<1024>(kAdjHbm);
  } else {
    if (block != 256 && block != 512 && block != 1024) return hipErrorInvalidValue;
    for (int w : {0, 8, 16, 32}) {
      if (block == 1024 && w == 0) continue;  // the general form has no 1024-thread kernel
      const void* k = block == 256 ? msc_kernel<256>(w)
                                   : block == 512 ? msc_kernel<512>(w) : msc_kernel<1024>(w);
      hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

hipError_t launch_argmax(const JobDev* jobs, int n_jobs, hipStream_t s) {
  hipLaunchKernelGGL(k_argmax, dim3(n_jobs), dim3(1024), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_gather(const void* buf, int layout, int R, int n_pad, int r, const int32_t* pos,
                         int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, s, buf, layout, R, n_pad, r,
                     pos, n, out);
  return hipGetLastError();
}

hipError_t launch_gather_states(const int8_t* src, int R, int n_pad, const int32_t* pos, int n,
                                int8_t* out, hipStream_t s) {
  const int64_t cnt = (int64_t)R * n;
  if (cnt <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_states, dim3(blocks_for(cnt, 256)), dim3(256), 0, s, src, R, n_pad, pos,
                     n, out);
  return hipGetLastError();
}

hipError_t launch_pt_init(const SwapDev& X, hipStream_t s) {
  const int n = X.K * X.n_sets;
  hipLaunchKernelGGL(k_pt_init, dim3(blocks_for(n, 256)), dim3(256), 0, s, X);
  return hipGetLastError();
}

hipError_t launch_swap(const SwapDev& X, int m, int32_t* clear8, hipStream_t s) {
  int n = X.n_sets * ((X.K - (m & 1)) / 2);
  if (clear8 && n < 8) n = 8;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_swap, dim3(blocks_for(n, 256)), dim3(256), 0, s, X, m, clear8);
  return hipGetLastError();
}

size_t houdayer_lds(int n, int n_pad, int n_adj, bool stage) {
  const size_t words = 4 * (size_t)((n_pad + 31) / 32);
  return sizeof(uint32_t) * words +
         (stage ? sizeof(int32_t) * (size_t)n_pad +
                      sizeof(uint16_t) * ((size_t)n_pad + 1 + (size_t)n_adj + (size_t)n)
                : 0);
}

hipError_t launch_houdayer(const ClusterDev& X, int m, int t, hipStream_t s) {
  const int wgs = X.n_pairs * (X.K - X.from);
  if (wgs <= 0) return hipSuccess;
  const size_t lds = houdayer_lds(X.n, X.n_pad, X.n_adj, X.stage != 0);
  if (lds > 48 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_houdayer,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) (void)hipGetLastError();  // advisory on this runtime
  }
  hipLaunchKernelGGL(k_houdayer, dim3(wgs), dim3(kClusterThreads), lds, s, X, m, t);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(count, 256)), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

}  // namespace ising
