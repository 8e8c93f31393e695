// device_types.h -- plain structs shared by the host runtime and the HIP
// kernels (no HIP or torch types).  All device arrays use the compiled
// problem's colour-major vertex order: each colour class occupies a run of
// positions padded to a multiple of four, so every aligned quadruple of
// positions is one random-number run ("group") of at most four same-colour
// vertices.
#pragma once
#include <stdint.h>

namespace ising {

// Per-group word: bits 0..27 = original id of the group's first vertex (the
// Philox counter word 0), bits 28..29 = number of real vertices - 1.
constexpr int32_t kGroupLeaderMask = 0x0FFFFFFF;
constexpr int kGroupCountShift = 28;

// Philox counter word 3 ("tag") of each purpose.
constexpr uint32_t kTagSweep = 0;
constexpr uint32_t kTagInit = 1;
constexpr uint32_t kTagSwap = 3;  // parallel tempering: (round, pair, set, 3)
constexpr uint32_t kTagCluster = 4;  // cluster moves: (round, temperature, set pair, 4)

// Threshold row length meaning "beta_t == 0: accept every move".
constexpr int32_t kAcceptAll = -1;

// Degree-4 group block, 12 words (48 bytes): words 0..7 hold the 16-bit LDS
// word indices of the 16 neighbour entries (slot j's four at 16-bit index
// 4j..4j+3, in label order: entry e of v is the neighbour u whose entry
// e XOR 1 is v), word 8 the group's first vertex, word 9 bit 4j+e set when entry e of
// slot j has w > 0; words 10 and 11 are zero.
constexpr int kDeg4BlockWords = 12;
// Multispin degree-4 form: 8 words (32 bytes) per group, the 16-bit
// element indices of slot j's four neighbours at 16-bit index 4j..4j+3,
// each naming the neighbour's element (even) or its complement (odd) so
// that the read element XOR the vertex's own is the bond's unsatisfied
// mask.  The state keeps element 2 i + 1 = NOT element 2 i.
constexpr int kDeg4MscBlockWords = 8;
// Multispin degree-4 form: at most this many groups of a lane's per sweep
// (sum over classes of ceil(class groups / (32 / W * threads))), so that the
// kernel's bit-sliced flip counters (8 planes) and sums of u (10 planes)
// cannot overflow: 4 x 63 < 2^8, 16 x 63 < 2^10.
constexpr int kMsc4MaxLaneIters = 63;

// FIELD path, degree-4 forms: a vertex's LDS word holds bond bits instead
// of a field.  Bit 0 is the spin bit b, bit 1 its complement, and bit
// kBondShift + e says whether the edge to entry e is satisfied
// (s_v J s_u = +1, J = -w).  The field follows: k = s h = 2 q - 4 for q
// satisfied bonds, and popc(word) = q + 1.  A flip XORs kBondFlipMask, a
// neighbour's flip one bond bit.
constexpr int kBondShift = 2;
constexpr int32_t kBondFlipMask = 0x3F;
// padding: popc 6, above every row's bound (at most 5), never flipped
constexpr int32_t kBondPadWord = 0x3F;
// Rows of the degree-4 forms, indexed by popc(word): [1..3] = 0xFFFFFFFF
// (k <= 0), [4], [5] = Tq - 1 of k = 2, 4 (0 beyond len), [6] = 0,
// [7] = the largest acceptable popc.
constexpr int kBondRowWords = 8;

// FIELD path: LDS words of one replica's state.  The degree-4 forms lay the
// state out in tiles of 64 groups, each tile holding its four slot planes
// of 64 words (position 4 g + j -> word 256 (g / 64) + 64 j + g mod 64), so
// the group count is rounded up to a multiple of 64.
constexpr int field_state_words(int n_pad) { return 4 * ((n_pad / 4 + 63) & ~63); }
constexpr int tile_word(int g, int j) { return ((g >> 6) << 8) + (j << 6) + (g & 63); }

// FIELD path: packed word of a padding slot.  Its k = s h = 2^30 - 1 is
// above every row's acceptable length (k never exceeds the problem's
// kmax < 2^29), so padding is never flipped.
constexpr int32_t kPadWord = 0x7FFFFFFF;

constexpr int kMaxReplicasPerBlock = 16;   // FIELD path
constexpr int kMaxFieldColours = 64;       // FIELD path: colour classes
constexpr int kMaxWordsPerBlock = 4;       // MSC path, general form (words of 32 replicas)
constexpr int kMaxThresholdRow = 1024;     // LDS paths stage <= this many
constexpr int kMaxLdsDegree = 255;         // LDS paths pack degrees in 8 bits

enum JobFlags : int32_t {
  kJobTrace = 1,      // write E after every sweep to trace[t*R + r]
  kJobInitGiven = 2,  // initial spins come from init_spins
  // FIELD degree-4 forms, between the segments of one tempering run: the
  // save area holds the units' bond words as they are in LDS, instead of
  // packed fields (written by a segment, read by the next one)
  kJobSaveBond = 4,
  kJobLoadBond = 8,
};

// One anneal of one problem for the persistent kernels.  Units of work are
// (job, replica block) pairs; a workgroup owns its block's replicas for all
// sweeps [t_begin, t_end) with the whole state resident in LDS.
struct JobDev {
  // graph, colour-major and padded
  const int32_t* row;    // [n_pad+1]
  const int32_t* adj;    // [2m] neighbour position
  const int32_t* wgt;    // [2m] MaxCut weight w (coupling J = -w)
  const uint32_t* adjm;  // [2m] (position << 1) | (w > 0), unit weights only
  const int2* aw;        // [2m] {neighbour position, w}
  const uint4* adj4;     // degree-4 graphs: [n_pad/4][3] group blocks (kDeg4Block*)
  const uint4* adj4m;    // degree-4 graphs, multispin form: [n_pad/4][2] (kDeg4MscBlockWords)
  const int32_t* grp;    // [n_pad/4] group words
  const int32_t* gbase;  // [n_pad/4] first adjacency entry of the group
  const uint32_t* gdeg;  // [n_pad/4] degrees of the group's four slots, 8 bits each
  const int32_t* cls;    // [2*C] first and end group of each class
  int32_t n_pad, n_colours;
  int32_t W;             // sum of weights
  int32_t M;             // edges
  // schedule
  const uint32_t* tq;    // thresholds minus one, rows back to back
  const int32_t* tq_off; // [S] row offsets into tq
  const int32_t* tq_len; // [S] row lengths, or kAcceptAll
  // FIELD: rows of 2 kw + 2 words indexed by the key x = 2 k - c (c = 1
  // for spin -1): [0] = 0xFFFFFFFF (k <= 0 always accepts), [x] for
  // x = 1..2 kw = Tq - 1 of k = ceil(x / 2), 0 beyond k = len,
  // [2 kw + 1] = twice the largest acceptable k (len, or kmax when beta = 0
  // and the row is all 0xFFFFFFFF)
  const uint32_t* tqp;   // [S][2 kw + 2]
  const uint32_t* tqb;   // FIELD degree-4 forms: [S][kBondRowWords]
  int32_t row_chunk;     // FIELD: sweeps whose rows are staged in LDS at once
  // parallel tempering: row of replica r is temp[r] for every sweep (the
  // rows are then one per temperature); null = row t for sweep t
  const int32_t* temp;
  // local fields b, position order [n_pad] (h = -sum w s + 2 b), or null
  const int32_t* bfield;
  int32_t S, t_begin, t_end, flags;
  int32_t kw;            // longest row (LDS row capacity)
  // run
  uint32_t seed_lo, seed_hi;
  int32_t R;             // replicas
  int32_t G;             // FIELD: replicas per block; MSC: words per block (general
                         // form) or replicas per block (degree-4 form: 8, 16, 32)
  int32_t adj_form;      // FIELD: this job's staged adjacency form (mixed launches)
  const int8_t* init_spins;  // [R][n_pad] +-1, positions order
  // state and outputs
  int32_t* save;         // FIELD: [R][n_pad] packed (h<<1)|bit; MSC: [nw][n_pad] words
  void* best;            // FIELD: int8 [R][n_pad]; MSC: uint32 [nw][n_pad]
  int32_t* best_cut;     // [R]
  int32_t* best_sweep;   // [R]
  int32_t* energy;       // [R]
  unsigned long long* accepts;  // [R]
  int32_t* trace;        // [S][R] when kJobTrace
  unsigned long long* argmax;   // [1] packed (best cut, replica) maximum
};

// Arguments of the per-colour-pass kernels (state in HBM, [position][R]).
struct PlainDev {
  const int32_t* row;
  const int32_t* adj;
  const int32_t* wgt;
  const int32_t* grp;
  int32_t n_pad, R, W, flags;
  const uint32_t* tq;
  const int32_t* tq_off;
  const int32_t* tq_len;
  const int32_t* temp;   // parallel tempering: row of replica r; null = row t
  const int32_t* bfield; // local fields [n_pad], or null
  uint32_t seed_lo, seed_hi;
  const int8_t* init_spins;  // [R][n_pad] or null
  int8_t* spins;         // [n_pad][R]
  int32_t* field;        // [n_pad][R]
  int8_t* best;          // [n_pad][R]
  int32_t* energy;       // [R]
  int32_t* eacc;         // [R] energy change of the current sweep
  int32_t* best_cut;     // [R]
  int32_t* best_sweep;   // [R]
  int32_t* snap;         // [R] last improving sweep (-1 = initial state)
  unsigned long long* accepts;  // [R]
  int32_t* trace;        // [S][R]
};

// Parallel tempering: the ladders of all sets and their exchange state.
// Replica r is in set r / K; slot[set K + k] is the replica at temperature
// k of its set and temp its inverse.  The exchange thresholds of pair
// (k, k+1) are a row of the flip-threshold form, for inverse temperature
// betas[k+1] - betas[k] and indexed by the cut difference q >= 1:
// tq[off[k] + q - 1] = Tq - 1 for q <= len[k] (Tq = 0 beyond), len[k] =
// kAcceptAll when the two betas are equal.
struct SwapDev {
  int32_t K, n_sets;
  uint32_t seed_lo, seed_hi;
  const int32_t* energy;   // [R] the run's current energies
  int32_t* temp;           // [R]
  int32_t* slot;           // [n_sets][K]
  long long* swaps;        // [n_sets][K-1] accepted exchanges
  const uint32_t* tq;
  const int32_t* off;      // [K-1]
  const int32_t* len;      // [K-1]
};

// Houdayer cluster moves of a tempering run (sets 2p and 2p+1 form pair
// p): one workgroup per (pair, temperature k >= from).  The replicas' state
// is either the FIELD save area (packed words (h << 1) | spin bit, [R][n_pad])
// or the PLAIN arrays (spins int8 and fields int32, [n_pad][R]).
struct ClusterDev {
  int32_t K, n_pairs, from;
  int32_t n, n_pad, R;
  int32_t n_adj;         // 2m adjacency entries
  int32_t stage;         // the parents, the position CSR and pos fit in LDS
                         // (the latter as 16-bit entries: n_pad, 2m < 2^16)
  int32_t unit;          // with stage: unit weights and n_pad < 2^15, so an
                         // entry's bit 15 can carry the sign of its weight
  uint32_t seed_lo, seed_hi;
  const int32_t* row;    // CSR over positions
  const int32_t* adj;
  const int32_t* wgt;
  const int32_t* grp;    // group words (real slots of a group)
  const int32_t* pos;    // [n] original id -> position
  const int32_t* slot;   // [n_sets][K] replica at each temperature
  int32_t* energy;       // [R]
  int32_t* packed;       // FIELD: [R][n_pad]; null on the plain path
  int8_t* spins;         // PLAIN: [n_pad][R]
  int32_t* field;        // PLAIN: [n_pad][R]
  int8_t* best;          // PLAIN: [n_pad][R] (pending lazy snapshots)
  int32_t* snap;         // PLAIN: [R] last improving sweep
  int32_t* queue;        // [workgroups][n_pad] union-find parents (when not staged)
  long long* moves;      // [n_pairs][K]
  long long* sites;      // [n_pairs][K]
};

// Layouts understood by the state gather kernel.
enum StateLayout : int32_t {
  kLayoutNR_I8 = 0,      // int8 [n_pad][R]
  kLayoutRN_I8 = 1,      // int8 [R][n_pad]
  kLayoutRN_Spin = 2,    // int32 packed [R][n_pad] -> bit 0 as +-1
  kLayoutRN_Field = 3,   // int32 packed [R][n_pad] -> value >> 1
  kLayoutNR_I32 = 4,     // int32 [n_pad][R]
  kLayoutWords = 5,      // uint32 [R/32][n_pad] -> bit r%32 as +-1
};

}  // namespace ising
