// anneal.cpp -- device memory, launch planning and the single-problem C ABI.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>

#include "runtime.h"

namespace ising {

// ---------------------------------------------------------------- memory
namespace {
std::mutex g_alloc_mu;
ising_alloc_fn g_alloc = nullptr;
ising_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
}  // namespace

int device_alloc(size_t bytes, DeviceBlock& out) {
  out = DeviceBlock();
  if (hipGetDevice(&out.device) != hipSuccess) {
    (void)hipGetLastError();
    set_error("no HIP device");
    return ISING_ERR_DEVICE;
  }
  ising_alloc_fn a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
    out.free_fn = g_free;
    out.ctx = g_alloc_ctx;
  }
  if (a) {
    out.ptr = a(bytes, out.device, out.ctx);
    if (!out.ptr || (reinterpret_cast<uintptr_t>(out.ptr) & 255u)) {
      set_error("the caller's allocator returned %s for %zu bytes",
                out.ptr ? "memory not aligned to 256 bytes" : "no memory", bytes);
      if (out.ptr) out.free_fn(out.ptr, bytes, out.device, out.ctx);
      out.ptr = nullptr;
      return ISING_ERR_NOMEM;
    }
  } else {
    out.free_fn = nullptr;
    hipError_t e = hipMalloc(&out.ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      out.ptr = nullptr;
      set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? ISING_ERR_NOMEM : ISING_ERR_DEVICE;
    }
  }
  out.bytes = bytes;
  return ISING_OK;
}

void device_free(DeviceBlock& b) {
  if (!b.ptr) return;
  DeviceGuard g(b.device);
  if (b.free_fn) {
    // the caller's allocator may hand the memory out again at once: let
    // every kernel that could still read it finish first
    (void)hipDeviceSynchronize();
    b.free_fn(b.ptr, b.bytes, b.device, b.ctx);
  } else {
    (void)hipFree(b.ptr);
  }
  b = DeviceBlock();
}

DeviceArena::~DeviceArena() { release(); }

void DeviceArena::release() {
  if (base && owned) device_free(block);
  block = DeviceBlock();
  base = nullptr;
  cap = used = 0;
  owned = true;
}

int DeviceArena::reserve(size_t bytes) {
  used = 0;
  if (bytes <= cap && base && owned) return ISING_OK;
  release();
  bytes = std::max<size_t>(bytes, 4096);
  IRET(device_alloc(bytes, block));
  device = block.device;
  base = static_cast<char*>(block.ptr);
  cap = bytes;
  ++generation;
  return ISING_OK;
}

RunBuffers::~RunBuffers() {
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
}

Launcher::~Launcher() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (staging) (void)hipHostFree(staging);
  if (staged) (void)hipEventDestroy(staged);
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  if (done) (void)hipEventDestroy(done);
}

int device_cu_count() {
  static std::mutex mu;
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
    cached[dev] = n;
  }
  return cached[dev];
}

size_t lds_budget(int path) {
  const size_t total = 160 * 1024;
  return total - (path == ISING_PATH_MSC ? kMscStaticLds : kFieldStaticLds);
}

int msc_planes(int max_deg) {
  int planes = 1;
  while ((1 << planes) <= max_deg) ++planes;
  return planes;
}

// ---------------------------------------------------------------- graph
int upload_graph(const HostGraph& g, DevGraph& d) {
  const size_t e2 = (size_t)(2 * g.m);
  size_t bytes = DeviceArena::span(sizeof(int32_t) * (g.n_pad + 1)) +
                 3 * DeviceArena::span(sizeof(int32_t) * e2) +
                 DeviceArena::span(sizeof(int2) * (e2 + 4)) +
                 3 * DeviceArena::span(sizeof(int32_t) * g.grp.size()) +
                 DeviceArena::span(sizeof(int32_t) * g.cls.size()) +
                 DeviceArena::span(sizeof(int32_t) * g.n) +
                 DeviceArena::span(sizeof(uint32_t) * g.adj4.size()) +
                 DeviceArena::span(sizeof(uint32_t) * g.adj4m.size()) +
                 DeviceArena::span(sizeof(int32_t) * (size_t)g.n_pad);
  IRET(d.arena.reserve(bytes));
  d.device = d.arena.device;
  d.row = d.arena.take<int32_t>(g.n_pad + 1);
  d.adj = d.arena.take<int32_t>(e2);
  d.wgt = d.arena.take<int32_t>(e2);
  d.adjm = d.arena.take<uint32_t>(e2);
  // four zero entries past the end: the FIELD kernel fetches four entries
  // per slot whatever the slot's degree
  d.aw = d.arena.take<int2>(e2 + 4);
  d.grp = d.arena.take<int32_t>(g.grp.size());
  d.gbase = d.arena.take<int32_t>(g.grp.size());
  d.gdeg = d.arena.take<uint32_t>(g.grp.size());
  d.cls = d.arena.take<int32_t>(g.cls.size());
  d.pos = d.arena.take<int32_t>(g.n);
  d.adj4 = g.adj4.empty() ? nullptr : d.arena.take<uint32_t>(g.adj4.size());
  d.adj4m = g.adj4m.empty() ? nullptr : d.arena.take<uint32_t>(g.adj4m.size());
  d.bf = d.arena.take<int32_t>((size_t)g.n_pad);
  ICHK(hipMemcpy(d.bf, g.bpos.data(), sizeof(int32_t) * (size_t)g.n_pad, hipMemcpyHostToDevice));
  if (d.adj4)
    ICHK(hipMemcpy(d.adj4, g.adj4.data(), sizeof(uint32_t) * g.adj4.size(), hipMemcpyHostToDevice));
  if (d.adj4m)
    ICHK(hipMemcpy(d.adj4m, g.adj4m.data(), sizeof(uint32_t) * g.adj4m.size(), hipMemcpyHostToDevice));
  ICHK(hipMemcpy(d.row, g.row.data(), sizeof(int32_t) * g.row.size(), hipMemcpyHostToDevice));
  if (e2) {
    ICHK(hipMemcpy(d.adj, g.adj.data(), sizeof(int32_t) * e2, hipMemcpyHostToDevice));
    ICHK(hipMemcpy(d.wgt, g.wgt.data(), sizeof(int32_t) * e2, hipMemcpyHostToDevice));
    ICHK(hipMemcpy(d.adjm, g.adjm.data(), sizeof(uint32_t) * e2, hipMemcpyHostToDevice));
    ICHK(hipMemcpy(d.aw, g.aw.data(), sizeof(int2) * e2, hipMemcpyHostToDevice));
  }
  {
    const int2 zero4[4] = {};
    ICHK(hipMemcpy(d.aw + e2, zero4, sizeof zero4, hipMemcpyHostToDevice));
  }
  ICHK(hipMemcpy(d.gbase, g.gbase.data(), sizeof(int32_t) * g.grp.size(), hipMemcpyHostToDevice));
  ICHK(hipMemcpy(d.gdeg, g.gdeg.data(), sizeof(uint32_t) * g.grp.size(), hipMemcpyHostToDevice));
  ICHK(hipMemcpy(d.grp, g.grp.data(), sizeof(int32_t) * g.grp.size(), hipMemcpyHostToDevice));
  ICHK(hipMemcpy(d.cls, g.cls.data(), sizeof(int32_t) * g.cls.size(), hipMemcpyHostToDevice));
  ICHK(hipMemcpy(d.pos, g.pos.data(), sizeof(int32_t) * g.n, hipMemcpyHostToDevice));
  return ISING_OK;
}

int upload_graph_once(const HostGraph& g, DevGraph& d) {
  if (d.device >= 0) return ISING_OK;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    set_error("no HIP device available");
    return ISING_ERR_DEVICE;
  }
  return upload_graph(g, d);
}

static int ensure_device(ising_problem* p) { return upload_graph_once(p->g, p->dg); }

// ---------------------------------------------------------------- planning
static bool pow2_upto(int x, int hi) { return x >= 1 && x <= hi && (x & (x - 1)) == 0; }

// Words of one FIELD row: entries for the keys x = 0 .. 2 kw and the bound.
static int field_row_words(const Table& t) { return 2 * std::max(t.kw, 1) + 2; }
// LDS stride budget of a row: either form (key rows, or the degree-4 forms'
// kBondRowWords) fits.
static int row_words_max(const Table& t) { return std::max(field_row_words(t), kBondRowWords); }

// FIELD rows are staged in chunks of up to 256 sweeps and about 8 KB.
static int row_chunk(const Table& t) {
  const int rw = row_words_max(t);
  return std::max(1, std::min(256, 2048 / rw));
}

// LDS of one unit: state words, a chunk of threshold rows, the class
// bounds and the group descriptors (group word, adjacency base, packed
// degrees).  The multispin kernel needs less (two rows, no class bounds).

// The multispin degree-4 form (c.G = 8, 16 or 32 replicas per unit): each
// state element next to its complement, and a chunk of degree-4 rows.
static bool msc4_config(const PersistentConfig& c) { return c.path == ISING_PATH_MSC && c.G >= 8; }

static size_t persistent_lds(const HostGraph& g, const Table& t, const PersistentConfig& c) {
  if (msc4_config(c))
    return (((size_t)field_state_words(g.n_pad) * (size_t)(c.G / 4) + 15) & ~(size_t)15) +
           sizeof(uint32_t) * (size_t)row_chunk(t) * kBondRowWords;
  const size_t rows = (size_t)row_chunk(t) * (size_t)row_words_max(t);
  return sizeof(int32_t) * ((size_t)c.G * field_state_words(g.n_pad) + rows + 2 * (size_t)g.C) +
         3 * sizeof(int32_t) * (size_t)(g.n_pad / 4);
}

// Rows of the FIELD kernel (JobDev::tqp): fixed stride so that a sweep's
// row is fetched without first reading its offset.  The kernel indexes a
// row by the key x = 2 k - c (c = 1 for spin -1, else 0), so entries
// 2 k - 1 and 2 k both hold the threshold of k.
size_t padded_rows(const Table& t) {
  return (size_t)t.S * (size_t)field_row_words(t);
}

void build_padded_rows(const Table& t, std::vector<uint32_t>& out) {
  const int kw = std::max(t.kw, 1), rw = field_row_words(t);
  out.assign(padded_rows(t), 0u);
  for (int s = 0; s < t.S; ++s) {
    uint32_t* row = out.data() + (size_t)s * rw;
    const int len = t.len[(size_t)s];
    row[0] = 0xFFFFFFFFu;
    if (len == kAcceptAll) {
      for (int x = 1; x <= 2 * kw; ++x) row[x] = 0xFFFFFFFFu;
      row[2 * kw + 1] = 2u * (uint32_t)t.kmax;
    } else {
      for (int x = 1; x <= 2 * len; ++x)
        row[x] = t.tq[(size_t)(t.off[(size_t)s] + (x + 1) / 2 - 1)];
      row[2 * kw + 1] = 2u * (uint32_t)len;
    }
  }
}

// Rows of the degree-4 forms (JobDev::tqb), indexed by the bond count plus
// one, c = popc(word) in 1..5, for k = 2 c - 6.
void build_bond_rows(const Table& t, std::vector<uint32_t>& out) {
  out.assign((size_t)t.S * kBondRowWords, 0u);
  for (int s = 0; s < t.S; ++s) {
    uint32_t* row = out.data() + (size_t)s * kBondRowWords;
    const int len = t.len[(size_t)s];
    for (int c = 0; c <= 3; ++c) row[c] = 0xFFFFFFFFu;  // k <= 0
    if (len == kAcceptAll) {
      row[4] = row[5] = 0xFFFFFFFFu;
      row[7] = 5;
    } else {
      const int32_t o = t.off[(size_t)s];
      row[4] = len >= 2 ? t.tq[(size_t)(o + 1)] : 0u;  // k = 2
      row[5] = len >= 4 ? t.tq[(size_t)(o + 3)] : 0u;  // k = 4
      row[7] = (uint32_t)std::min(5, (len + 6) / 2);   // 2 c - 6 <= len
    }
  }
}

// Staged adjacency forms of the FIELD kernel (16-bit entries).
constexpr int kFormHbm = 0, kFormCsr = 1, kFormDeg4 = 2;
constexpr int kFormPerJob = 3;   // a launch whose jobs use different forms
constexpr int kFormHbmDeg4 = 4;  // degree-4 blocks read from HBM (too large for LDS)

// Extra LDS of a staged form: up to 12 bytes that align the entries to 16
// bytes, then the CSR form's 2m entries, a gap word and the per-wave flip
// lists (256 entries per wave of the largest block), or the degree-4 form's
// 48-byte group blocks.
static size_t adjacency_lds(const HostGraph& g, int form) {
  if (form == kFormHbmDeg4) return 0;
  if (form == kFormDeg4) return 12 + 4 * kDeg4BlockWords * (size_t)(g.n_pad / 4);
  return 12 + 4 * (size_t)g.m + 4 + (size_t)(1024 / 64) * 256 * 4;
}
static bool adjacency_fits(const HostGraph& g, int form) {
  // the degree-4 forms' bond words carry no field term
  if (form == kFormHbmDeg4) return !g.adj4.empty() && !g.fields;
  if (form == kFormDeg4) return !g.adj4.empty() && !g.fields && g.n_pad < (1 << 15);
  return g.unit && g.n_pad < (1 << 15) && 2 * g.m < (1 << 17) && g.max_deg <= 255;
}
// The adjacency form that tuning value `adj` (0 decide, 1 LDS, 2 HBM
// pairs, 3 LDS in CSR form, 4 degree-4 blocks from HBM) gives g: the
// degree-4 form staged in LDS when it fits, else its blocks read from HBM,
// else the CSR form staged; kFormHbm ({position, w} pairs) otherwise.  For
// adj = 1 and 3 the caller refuses a result that is not staged.
static int staged_form(const HostGraph& g, const Table& t, const PersistentConfig& c) {
  if (c.path != ISING_PATH_FIELD || c.adj == 2) return kFormHbm;
  if (c.adj == 4) return adjacency_fits(g, kFormHbmDeg4) ? kFormHbmDeg4 : kFormHbm;
  const size_t base = persistent_lds(g, t, c);
  const bool fits_deg4 = adjacency_fits(g, kFormDeg4) &&
                         base + adjacency_lds(g, kFormDeg4) <= lds_budget(c.path);
  const bool fits_csr = adjacency_fits(g, kFormCsr) &&
                        base + adjacency_lds(g, kFormCsr) <= lds_budget(c.path);
  if (c.adj == 3) return fits_csr ? kFormCsr : kFormHbm;
  if (fits_deg4) return kFormDeg4;
  if (c.adj == 0 && adjacency_fits(g, kFormHbmDeg4)) return kFormHbmDeg4;
  return fits_csr ? kFormCsr : kFormHbm;
}
static bool form_in_lds(int form) { return form == kFormCsr || form == kFormDeg4; }

int check_config(const HostGraph& g, const Table& t, int R, const PersistentConfig& c) {
  (void)R;
  if (c.path == ISING_PATH_PLAIN) return ISING_OK;
  if (c.path != ISING_PATH_FIELD && c.path != ISING_PATH_MSC) {
    set_error("unknown path %d", c.path);
    return ISING_ERR_INVALID;
  }
  if (c.block != 256 && c.block != 512 && c.block != 1024) {
    set_error("block_threads must be 256, 512 or 1024");
    return ISING_ERR_INVALID;
  }
  if (msc4_config(c)) {
    if (c.G != 8 && c.G != 16 && c.G != 32) {
      set_error("the multispin degree-4 form takes 8, 16 or 32 replicas per block");
      return ISING_ERR_INVALID;
    }
  } else {
    const int gmax = c.path == ISING_PATH_FIELD ? kMaxReplicasPerBlock : kMaxWordsPerBlock;
    if (!pow2_upto(c.G, gmax) || c.block / c.G < 64) {
      set_error("replicas_per_block %d invalid for %d threads", c.G, c.block);
      return ISING_ERR_INVALID;
    }
  }
  if (c.adj < 0 || c.adj > 4) {
    set_error("adjacency mode %d invalid", c.adj);
    return ISING_ERR_INVALID;
  }
  if (c.adj == 4 && (c.path != ISING_PATH_FIELD || !adjacency_fits(g, kFormHbmDeg4))) {
    set_error("the degree-4 adjacency form needs unit weights, every vertex of degree 4, "
              "at most 2^16 positions and no local fields");
    return ISING_ERR_UNSUPPORTED;
  }
  if ((c.adj == 1 || c.adj == 3) && !form_in_lds(staged_form(g, t, c))) {
    set_error("the adjacency cannot be staged in LDS for this problem");
    return ISING_ERR_UNSUPPORTED;
  }
  if (c.path == ISING_PATH_FIELD && g.C > kMaxFieldColours) {
    set_error("the field path supports at most %d colour classes", kMaxFieldColours);
    return ISING_ERR_UNSUPPORTED;
  }
  if (c.path == ISING_PATH_MSC) {
    if (g.fields) {
      set_error("the multispin path has no local field term");
      return ISING_ERR_UNSUPPORTED;
    }
    if (!g.unit) {
      set_error("the multispin path needs all |w| == 1");
      return ISING_ERR_UNSUPPORTED;
    }
    if (g.max_deg > 31) {
      set_error("the multispin path supports degree <= 31");
      return ISING_ERR_UNSUPPORTED;
    }
    if (msc4_config(c)) {
      if (g.adj4m.empty()) {
        set_error("the multispin degree-4 form needs every vertex of degree 4 and at most "
                  "2^15 padded positions");
        return ISING_ERR_UNSUPPORTED;
      }
      if (g.C > kMaxFieldColours) {
        set_error("the multispin degree-4 form supports at most %d colour classes", kMaxFieldColours);
        return ISING_ERR_UNSUPPORTED;
      }
      // groups a lane meets per sweep bound the kernel's counter planes
      const int per_iter = (32 / c.G) * c.block;
      int its = 0;
      for (int k = 0; k < g.C; ++k)
        its += (g.cls[(size_t)(2 * k + 1)] - g.cls[(size_t)(2 * k)] + per_iter - 1) / per_iter;
      if (its > kMsc4MaxLaneIters) {
        set_error("the multispin degree-4 form with %d replicas and %d threads per block takes at "
                  "most %d groups per lane and sweep (this problem needs %d)",
                  c.G, c.block, kMsc4MaxLaneIters, its);
        return ISING_ERR_UNSUPPORTED;
      }
    } else if (c.block == 1024) {
      set_error("the general multispin form runs 256 or 512 threads");
      return ISING_ERR_INVALID;
    }
  }
  if (g.max_deg > kMaxLdsDegree) {
    set_error("degrees above %d need the plain path", kMaxLdsDegree);
    return ISING_ERR_UNSUPPORTED;
  }
  if (t.kw > kMaxThresholdRow) {
    set_error("threshold rows longer than %d need the plain path", kMaxThresholdRow);
    return ISING_ERR_UNSUPPORTED;
  }
  if (c.path == ISING_PATH_FIELD && (int64_t)padded_rows(t) > kMaxTableEntries) {
    set_error("sweeps x (row length + 2) above 2^26 need the plain path");
    return ISING_ERR_UNSUPPORTED;
  }
  if (persistent_lds(g, t, c) > lds_budget(c.path)) {
    set_error("problem does not fit the %zu-byte LDS budget with %d replica(s) per block",
              lds_budget(c.path), c.G);
    return ISING_ERR_UNSUPPORTED;
  }
  return ISING_OK;
}

PersistentConfig heuristic_config(const HostGraph& g, const Table& t, int R) {
  PersistentConfig c;
  c.path = ISING_PATH_FIELD;
  c.G = 1;
  c.block = 1024;
  const int cus = std::max(device_cu_count(), 1);
  // One replica per block, with about one thread per group of a colour
  // class: smaller blocks leave LDS for more resident blocks per CU.
  const int per_class = std::max(1, g.n_pad / 4 / std::max(g.C, 1));
  while (c.block > 256 && per_class * 2 <= c.block) c.block /= 2;
  // Several replicas per block only when one replica leaves most of the
  // block idle and replicas are plentiful, so that the unit count stays
  // above the CU count.
  while (c.G < kMaxReplicasPerBlock && c.block / c.G / 2 >= 64 && per_class * 2 <= c.block / c.G &&
         (R / (2 * c.G)) >= 2 * cus) {
    PersistentConfig n = c;
    n.G *= 2;
    if (persistent_lds(g, t, n) > lds_budget(n.path)) break;
    c = n;
  }
  if (check_config(g, t, R, c) != ISING_OK) c.path = ISING_PATH_PLAIN;
  return c;
}

// ---------------------------------------------------------------- run state
size_t run_bytes(const HostGraph& g, const Table& table, int R, const PersistentConfig& cfg,
                 bool trace, bool init_given) {
  const size_t np = (size_t)g.n_pad, RR = (size_t)R;
  const size_t nw = (size_t)(R + 31) / 32;
  const size_t S = (size_t)table.S;
  const bool plain = cfg.path == ISING_PATH_PLAIN, msc = cfg.path == ISING_PATH_MSC;
  const size_t best_bytes = msc ? sizeof(uint32_t) * nw * np : np * RR;
  const size_t save_bytes = plain ? 0 : (msc ? sizeof(uint32_t) * nw * np : sizeof(int32_t) * RR * np);
  return DeviceArena::span(best_bytes) + DeviceArena::span(save_bytes) +
         (plain ? DeviceArena::span(np * RR) + DeviceArena::span(sizeof(int32_t) * np * RR) : 0) +
         5 * DeviceArena::span(sizeof(int32_t) * RR) +
         DeviceArena::span(sizeof(unsigned long long) * RR) +
         DeviceArena::span(sizeof(unsigned long long)) +
         (trace ? DeviceArena::span(sizeof(int32_t) * S * RR) : 0) +
         DeviceArena::span(sizeof(int32_t) * (size_t)g.n) +
         DeviceArena::span(sizeof(uint32_t) * table.tq.size()) +
         2 * DeviceArena::span(sizeof(int32_t) * S) + (init_given ? DeviceArena::span(RR * np) : 0) +
         (cfg.path == ISING_PATH_FIELD ? DeviceArena::span(sizeof(uint32_t) * padded_rows(table)) : 0) +
         (cfg.path == ISING_PATH_FIELD || msc
              ? DeviceArena::span(sizeof(uint32_t) * kBondRowWords * S)
              : 0) +
         DeviceArena::span(sizeof(JobDev));
}

int prepare_buffers(RunBuffers& b, const HostGraph& g, const Table& table, int R,
                    const PersistentConfig& cfg, hipStream_t stream, bool trace,
                    const int8_t* init, char* pool) {
  if (b.valid && b.stream) (void)hipStreamSynchronize(b.stream);
  b.valid = false;
  const size_t np = (size_t)g.n_pad, RR = (size_t)R;
  const int nw = (R + 31) / 32;
  const int S = table.S;
  const bool plain = cfg.path == ISING_PATH_PLAIN, msc = cfg.path == ISING_PATH_MSC;
  const bool init_given = init != nullptr;
  const size_t bytes = run_bytes(g, table, R, cfg, trace, init_given);
  if (pool) {
    int dev = -1;
    ICHK(hipGetDevice(&dev));
    b.arena.adopt(pool, bytes, dev);
  } else {
    IRET(b.arena.reserve(bytes));
  }
  b.R = R;
  b.S = S;
  b.path = cfg.path;
  b.G = cfg.G;
  b.block = cfg.block;
  b.nw = nw;
  b.trace = trace;
  b.best = msc ? (void*)b.arena.take<uint32_t>(nw * np) : (void*)b.arena.take<int8_t>(np * RR);
  b.save = plain ? nullptr : b.arena.take<int32_t>(msc ? nw * np : RR * np);
  b.spins = plain ? b.arena.take<int8_t>(np * RR) : nullptr;
  b.field = plain ? b.arena.take<int32_t>(np * RR) : nullptr;
  b.best_cut = b.arena.take<int32_t>(RR);
  b.best_sweep = b.arena.take<int32_t>(RR);
  b.energy = b.arena.take<int32_t>(RR);
  b.eacc = b.arena.take<int32_t>(RR);
  b.snap = b.arena.take<int32_t>(RR);
  b.accepts = b.arena.take<unsigned long long>(RR);
  b.argmax = b.arena.take<unsigned long long>(1);
  b.trace_buf = trace ? b.arena.take<int32_t>((size_t)S * RR) : nullptr;
  b.gather = b.arena.take<int32_t>((size_t)g.n);
  b.tq = b.arena.take<uint32_t>(table.tq.size());
  b.tq_off = b.arena.take<int32_t>((size_t)S);
  b.tq_len = b.arena.take<int32_t>((size_t)S);
  b.tqp = cfg.path == ISING_PATH_FIELD ? b.arena.take<uint32_t>(padded_rows(table)) : nullptr;
  b.tqb = cfg.path == ISING_PATH_FIELD || msc ? b.arena.take<uint32_t>((size_t)kBondRowWords * S)
                                              : nullptr;
  b.init_dev = init_given ? b.arena.take<int8_t>(RR * np) : nullptr;
  b.job_dev = b.arena.take<JobDev>(1);
  if (plain) {
    b.layout_best = kLayoutNR_I8;
    b.layout_final = kLayoutNR_I8;
    b.layout_field = kLayoutNR_I32;
  } else if (msc) {
    b.layout_best = kLayoutWords;
    b.layout_final = kLayoutWords;
    b.layout_field = -1;
  } else {
    b.layout_best = kLayoutRN_I8;
    b.layout_final = kLayoutRN_Spin;
    b.layout_field = kLayoutRN_Field;
  }
  if (!b.ev0) ICHK(hipEventCreate(&b.ev0));
  if (!b.ev1) ICHK(hipEventCreate(&b.ev1));
  b.stream = stream;
  // The tables are uploaded unless this same table already sits at these
  // addresses of this same arena (a pool's memory is always rewritten).
  const void* at = b.tqp ? (const void*)b.tqp : b.tqb ? (const void*)b.tqb : (const void*)b.tq;
  const bool resident = !pool && table.id != 0 && b.up_table == table.id &&
                        b.up_generation == b.arena.generation && b.up_at == at;
  if (!resident) {
    // the host copy outlives the asynchronous uploads (until the next run)
    b.table = table;
    ICHK(hipMemcpyAsync(b.tq, b.table.tq.data(), sizeof(uint32_t) * b.table.tq.size(),
                        hipMemcpyHostToDevice, stream));
    ICHK(hipMemcpyAsync(b.tq_off, b.table.off.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice,
                        stream));
    ICHK(hipMemcpyAsync(b.tq_len, b.table.len.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice,
                        stream));
    if (b.tqp) {
      build_padded_rows(b.table, b.tqp_host);
      ICHK(hipMemcpyAsync(b.tqp, b.tqp_host.data(), sizeof(uint32_t) * b.tqp_host.size(),
                          hipMemcpyHostToDevice, stream));
    }
    if (b.tqb) {
      build_bond_rows(b.table, b.tqb_host);
      ICHK(hipMemcpyAsync(b.tqb, b.tqb_host.data(), sizeof(uint32_t) * b.tqb_host.size(),
                          hipMemcpyHostToDevice, stream));
    }
    b.up_table = table.id;
    b.up_generation = b.arena.generation;
    b.up_at = at;
  }
  if (init_given) {
    std::vector<int8_t> perm(RR * np, 1);
    for (size_t r = 0; r < RR; ++r)
      for (int32_t v = 0; v < g.n; ++v)
        perm[r * np + (size_t)g.pos[(size_t)v]] = init[r * (size_t)g.n + (size_t)v];
    // synchronous: the temporary buffer dies at return
    ICHK(hipMemcpy(b.init_dev, perm.data(), RR * np, hipMemcpyHostToDevice));
  }
  return ISING_OK;
}

int prepare_run(ising_problem* p, const Table& table, int R, const PersistentConfig& cfg,
                hipStream_t stream) {
  if (p->init_R > 0 && p->init_R != R) {
    set_error("initial states were given for %d replicas, anneal asks %d", p->init_R, R);
    return ISING_ERR_STATE;
  }
  return prepare_buffers(p->run, p->g, table, R, cfg, stream, p->trace,
                         p->init_R > 0 ? p->init.data() : nullptr, nullptr);
}

JobDev make_job(const HostGraph& g, const DevGraph& d, const RunBuffers& b, int R, uint64_t seed,
                int t_begin, int t_end, const PersistentConfig& cfg) {
  const Table& table = b.table;
  JobDev J;
  memset(&J, 0, sizeof J);
  J.row = d.row;
  J.adj = d.adj;
  J.wgt = d.wgt;
  J.adjm = d.adjm;
  J.adj4 = reinterpret_cast<const uint4*>(d.adj4);
  J.adj4m = reinterpret_cast<const uint4*>(d.adj4m);
  J.aw = d.aw;
  J.grp = d.grp;
  J.gbase = d.gbase;
  J.gdeg = d.gdeg;
  J.cls = d.cls;
  J.n_pad = g.n_pad;
  J.n_colours = g.C;
  J.W = (int32_t)g.W;
  J.M = (int32_t)g.m;
  J.tq = b.tq;
  J.tq_off = b.tq_off;
  J.tq_len = b.tq_len;
  J.tqp = b.tqp;
  J.tqb = b.tqb;
  J.row_chunk = row_chunk(table);
  J.S = table.S;
  J.t_begin = t_begin;
  J.t_end = t_end;
  J.flags = (b.trace ? kJobTrace : 0) | (b.init_dev ? kJobInitGiven : 0);
  J.kw = std::max(table.kw, 1);
  J.seed_lo = (uint32_t)seed;
  J.seed_hi = (uint32_t)(seed >> 32);
  J.R = R;
  J.G = cfg.G;
  J.init_spins = b.init_dev;
  J.save = b.save;
  J.best = b.best;
  J.best_cut = b.best_cut;
  J.best_sweep = b.best_sweep;
  J.energy = b.energy;
  J.accepts = b.accepts;
  J.trace = b.trace_buf;
  J.argmax = b.argmax;
  J.bfield = g.fields ? d.bf : nullptr;
  return J;
}

// ---------------------------------------------------------------- persistent
int temper_max_group(const Table& t) { return row_chunk(t); }

int plan_persistent(const std::vector<JobSpec>& specs, const PersistentConfig& cfg,
                    PersistentPlan& P) {
  const int n_jobs = (int)specs.size();
  std::vector<JobDev>& jobs = P.jobs;
  jobs.assign((size_t)n_jobs, JobDev());
  struct U {
    double cost;
    int job, block;
  };
  std::vector<U> all;
  // Each FIELD job stages the best adjacency form that fits it (degree-4,
  // then CSR), else reads HBM; a launch whose jobs differ runs the kernel
  // that picks the form per job.
  std::vector<int> forms((size_t)n_jobs, kFormHbm);
  size_t lds = 0, lds_staged = 0;
  int planes = 1;
  for (int j = 0; j < n_jobs; ++j) {
    const JobSpec& s = specs[(size_t)j];
    jobs[(size_t)j] = make_job(*s.g, *s.dg, *s.b, s.R, s.seed, s.t_begin, s.t_end, cfg);
    const size_t own = persistent_lds(*s.g, s.b->table, cfg);
    lds = std::max(lds, own);
    const int f = staged_form(*s.g, s.b->table, cfg);
    if ((cfg.adj == 1 || cfg.adj == 3) && !form_in_lds(f)) {
      set_error("the adjacency of problem %d cannot be staged in LDS", j);
      return ISING_ERR_UNSUPPORTED;
    }
    forms[(size_t)j] = f;
    lds_staged = std::max(lds_staged, own + (form_in_lds(f) ? adjacency_lds(*s.g, f) : 0));
    planes = std::max(planes, msc_planes(s.g->max_deg));
    const int per = msc4_config(cfg) ? cfg.G : cfg.path == ISING_PATH_MSC ? 32 * cfg.G : cfg.G;
    const int nb = (s.R + per - 1) / per;
    const double cost = (double)s.g->n_pad * (s.t_end - s.t_begin) * per + 1.0;
    for (int k = 0; k < nb; ++k) all.push_back(U{cost, j, k});
  }
  if (lds > lds_budget(cfg.path)) {
    set_error("batch does not fit the LDS budget");
    return ISING_ERR_UNSUPPORTED;
  }
  // Longest processing time first, over eight lists (one per XCD).  With
  // many jobs, all units of a job go to one list, so that its graph and
  // tables are read through one XCD's L2 only (the lists are balanced by
  // job); with few jobs the units spread over all lists.
  std::stable_sort(all.begin(), all.end(), [](const U& a, const U& b) { return a.cost > b.cost; });
  std::vector<std::vector<int2>> lists(8);
  double load[8] = {0};
  auto least = [&]() {
    int best = 0;
    for (int i = 1; i < 8; ++i)
      if (load[i] < load[best]) best = i;
    return best;
  };
  if (n_jobs >= 16) {
    std::vector<double> job_cost((size_t)n_jobs, 0.0);
    for (const U& u : all) job_cost[(size_t)u.job] += u.cost;
    std::vector<int> order((size_t)n_jobs);
    for (int j = 0; j < n_jobs; ++j) order[(size_t)j] = j;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return job_cost[(size_t)a] > job_cost[(size_t)b]; });
    std::vector<int> list_of((size_t)n_jobs, 0);
    for (int j : order) {
      const int best = least();
      load[best] += job_cost[(size_t)j];
      list_of[(size_t)j] = best;
    }
    for (const U& u : all) lists[(size_t)list_of[(size_t)u.job]].push_back(make_int2(u.job, u.block));
  } else {
    for (const U& u : all) {
      const int best = least();
      load[best] += u.cost;
      lists[(size_t)best].push_back(make_int2(u.job, u.block));
    }
  }
  std::vector<int2>& units = P.units;
  units.clear();
  P.list_off[0] = 0;
  for (int i = 0; i < 8; ++i) {
    units.insert(units.end(), lists[(size_t)i].begin(), lists[(size_t)i].end());
    P.list_off[i + 1] = (int32_t)units.size();
  }
  const int n_units = (int)units.size();
  P.grid = 0;
  if (n_units == 0) return ISING_OK;

  const int cus = std::max(device_cu_count(), 1);
  if (cfg.path == ISING_PATH_MSC) {
    // the multispin kernels read their adjacency from HBM; the form slot
    // carries the width (0 = the general form)
    const int width = msc4_config(cfg) ? cfg.G : 0;
    if (set_persistent_lds_limit(cfg.path, cfg.block, lds) != hipSuccess) (void)hipGetLastError();
    const int occ = persistent_occupancy(cfg.path, cfg.block, width, lds);
    if (occ <= 0) {
      set_error("persistent kernel cannot be resident with %zu bytes of LDS", lds);
      return ISING_ERR_UNSUPPORTED;
    }
    P.lds = lds;
    P.form = width;
    P.planes = planes;
    P.grid = std::min(n_units, cus * occ);
    return ISING_OK;
  }
  int form = forms.empty() ? kFormHbm : forms[0];
  bool staged = false;
  for (int f : forms) {
    if (f != form) form = kFormPerJob;
    staged = staged || form_in_lds(f);
  }
  if (cfg.adj == 0 && staged) {
    // stage only when that does not cost concurrency the units could use
    const int occ_adj = persistent_occupancy(cfg.path, cfg.block, form, lds_staged);
    const int occ_plain = persistent_occupancy(cfg.path, cfg.block, kFormHbm, lds);
    if (!(occ_adj > 0 && (occ_adj == occ_plain || (int64_t)n_units <= (int64_t)cus * occ_adj))) {
      // keep the forms that need no LDS
      staged = false;
      form = -1;
      for (size_t j = 0; j < forms.size(); ++j) {
        const JobSpec& s = specs[j];
        if (form_in_lds(forms[j]))
          forms[j] = adjacency_fits(*s.g, kFormHbmDeg4) ? kFormHbmDeg4 : kFormHbm;
        form = form < 0 || form == forms[j] ? forms[j] : kFormPerJob;
      }
    }
  }
  if (staged) lds = lds_staged;
  for (int j = 0; j < n_jobs; ++j) jobs[(size_t)j].adj_form = forms[(size_t)j];
  // raising the dynamic LDS limit is advisory on this runtime
  if (set_persistent_lds_limit(cfg.path, cfg.block, lds) != hipSuccess) (void)hipGetLastError();
  const int occ = persistent_occupancy(cfg.path, cfg.block, form, lds);
  if (occ <= 0) {
    set_error("persistent kernel cannot be resident with %zu bytes of LDS", lds);
    return ISING_ERR_UNSUPPORTED;
  }
  P.lds = lds;
  P.form = form;
  P.planes = planes;
  P.grid = std::min(n_units, cus * occ);
  return ISING_OK;
}

int run_persistent(Launcher& L, const std::vector<JobSpec>& specs, const PersistentConfig& cfg,
                   hipStream_t stream, bool use_graph, const TemperPlan* pt) {
  const int n_jobs = (int)specs.size();
  if (pt && (n_jobs != 1 || cfg.path != ISING_PATH_FIELD || cfg.G > row_chunk(specs[0].b->table))) {
    set_error("tempering runs one FIELD job with at most %d replicas per block",
              n_jobs == 1 ? row_chunk(specs[0].b->table) : 0);
    return ISING_ERR_UNSUPPORTED;
  }
  // segments of the sweeps: one launch each (tempering: up to every
  // exchange round), else the jobs' own ranges in one launch
  std::vector<int2> segs;
  if (pt) {
    for (int t0 = 0; t0 < pt->S; t0 += pt->P) segs.push_back(make_int2(t0, std::min(pt->S, t0 + pt->P)));
  } else {
    segs.push_back(make_int2(-1, -1));
  }
  const int n_segs = (int)segs.size();
  PersistentPlan plan;
  IRET(plan_persistent(specs, cfg, plan));
  std::vector<JobDev>& jobs = plan.jobs;
  const std::vector<int2>& units = plan.units;
  const int32_t* list_off = plan.list_off;
  const int n_units = (int)units.size();
  if (n_units == 0) return ISING_OK;
  const size_t lds = plan.lds;
  const int form = plan.form, planes = plan.planes;
  if (pt) {
    // one copy of the job per segment
    JobDev base = jobs[0];
    base.temp = pt->swap->temp;
    jobs.assign((size_t)n_segs, base);
    // Between segments only the exchange kernel runs, and it reads
    // energies: a degree-4 form keeps its bond words in the save area from
    // one segment to the next, and only the last segment saves packed
    // fields.  Cluster moves read the packed form after every round.
    const bool bond = !pt->cluster && (form == kFormDeg4 || form == kFormHbmDeg4 ||
                                        (form == kFormPerJob &&
                                         (base.adj_form == kFormDeg4 || base.adj_form == kFormHbmDeg4)));
    for (int i = 0; i < n_segs; ++i) {
      JobDev& J = jobs[(size_t)i];
      J.t_begin = segs[(size_t)i].x;
      J.t_end = segs[(size_t)i].y;
      if (bond && i > 0) J.flags |= kJobLoadBond;
      if (bond && i + 1 < n_segs) J.flags |= kJobSaveBond;
    }
  }
  const int n_dev_jobs = (int)jobs.size();

  // The jobs, units and list cursors on the device are shared by every
  // launch of this launcher.  A launch on another stream must not rewrite
  // them while an earlier one still claims units, so this stream first
  // waits for the previous launch (on the same stream the wait is already
  // implied by stream order).
  if (L.done_recorded) ICHK(hipStreamWaitEvent(stream, L.done, 0));
  // device and pinned staging buffers (a reallocation frees the old
  // device buffers after a device synchronisation)
  if (L.jobs_cap < (size_t)n_dev_jobs || L.units_cap < (size_t)n_units || !L.arena.base) {
    L.jobs_cap = std::max<size_t>(n_dev_jobs, 16);
    L.units_cap = std::max<size_t>(n_units, 1024);
    size_t bytes = DeviceArena::span(sizeof(JobDev) * L.jobs_cap) +
                   DeviceArena::span(sizeof(int2) * L.units_cap) + 2 * DeviceArena::span(64);
    IRET(L.arena.reserve(bytes));
    L.jobs_d = L.arena.take<JobDev>(L.jobs_cap);
    L.units_d = L.arena.take<int2>(L.units_cap);
    L.list_off_d = L.arena.take<int32_t>(16);
    L.ctr_d = L.arena.take<int32_t>(16);
  }
  const size_t stage_bytes = sizeof(JobDev) * n_dev_jobs + sizeof(int2) * n_units + sizeof(plan.list_off);
  if (!L.staged) ICHK(hipEventCreateWithFlags(&L.staged, hipEventDisableTiming));
  (void)hipEventSynchronize(L.staged);  // the previous upload has left the buffer
  if (L.staging_cap < stage_bytes) {
    if (L.staging) (void)hipHostFree(L.staging);
    L.staging = nullptr;
    L.staging_cap = std::max<size_t>(stage_bytes, 1 << 16);
    ICHK(hipHostMalloc((void**)&L.staging, L.staging_cap, hipHostMallocDefault));
  }
  char* sp = L.staging;
  const size_t jb = sizeof(JobDev) * n_dev_jobs;
  memcpy(sp, jobs.data(), jb);
  memcpy(sp + jb, units.data(), sizeof(int2) * n_units);
  memcpy(sp + jb + sizeof(int2) * n_units, list_off, sizeof(plan.list_off));
  ICHK(hipMemcpyAsync(L.jobs_d, sp, jb, hipMemcpyHostToDevice, stream));
  ICHK(hipMemcpyAsync(L.units_d, sp + jb, sizeof(int2) * n_units, hipMemcpyHostToDevice, stream));
  ICHK(hipMemcpyAsync(L.list_off_d, sp + jb + sizeof(int2) * n_units, sizeof(plan.list_off),
                      hipMemcpyHostToDevice, stream));
  ICHK(hipEventRecord(L.staged, stream));

  LaunchPersistent lp;
  lp.jobs = L.jobs_d;
  lp.units = L.units_d;
  lp.list_off = L.list_off_d;
  lp.ctr = L.ctr_d;
  lp.grid = plan.grid;
  lp.lds_bytes = lds;
  lp.planes = planes;
  lp.adj = cfg.path == ISING_PATH_MSC ? 0 : form;
  lp.width = cfg.path == ISING_PATH_MSC ? form : 0;

  // An exchange round also clears the list cursors for the next segment.
  auto enqueue = [&](hipStream_t s) -> hipError_t {
    bool cleared = false;
    for (int i = 0; i < n_segs; ++i) {
      hipError_t e = hipSuccess;
      if (!cleared) e = launch_fill_i32(L.ctr_d, 0, 8, s);
      if (e != hipSuccess) return e;
      LaunchPersistent li = lp;
      li.jobs = L.jobs_d + (pt ? i : 0);
      e = cfg.path == ISING_PATH_MSC ? launch_msc(li, cfg.block, s) : launch_field(li, cfg.block, s);
      if (e != hipSuccess) return e;
      cleared = false;
      if (pt && segs[(size_t)i].y % pt->P == 0) {
        const int m = segs[(size_t)i].y / pt->P - 1;
        if (pt->cluster) {
          e = launch_houdayer(*pt->cluster, m, segs[(size_t)i].y - 1, s);
          if (e != hipSuccess) return e;
        }
        e = launch_swap(*pt->swap, m, L.ctr_d, s);
        if (e != hipSuccess) return e;
        cleared = true;
      }
    }
    return launch_argmax(L.jobs_d, n_jobs, s);
  };

  if (!L.ev0) ICHK(hipEventCreate(&L.ev0));
  if (!L.ev1) ICHK(hipEventCreate(&L.ev1));
  ICHK(hipEventRecord(L.ev0, stream));
  if (use_graph && stream) {
    char key[512];
    int kl = snprintf(key, sizeof key, "%d/%d/%d/%d/%d/%zu/%d/%d/%d/%p", cfg.path, cfg.block, cfg.G,
                      planes, form, lds, lp.grid, n_jobs, n_units, (void*)L.arena.base);
    if (pt) {
      // the exchange launches carry their arguments by value
      const SwapDev& X = *pt->swap;
      kl += snprintf(key + kl, sizeof key - (size_t)kl, "/pt/%d/%d/%d/%d/%u/%u/%p/%p/%p/%p/%p/%p/%p",
                     pt->S, pt->P, X.K, X.n_sets, X.seed_lo, X.seed_hi, (const void*)X.energy,
                     (void*)X.temp, (void*)X.slot, (void*)X.swaps, (const void*)X.tq,
                     (const void*)X.off, (const void*)X.len);
      if (pt->cluster) {
        const ClusterDev& Y = *pt->cluster;
        snprintf(key + kl, sizeof key - (size_t)kl, "/cl/%d/%d/%d/%p/%p/%p/%p", Y.from, Y.n_pairs,
                 Y.stage, (void*)Y.queue, (void*)Y.moves, (void*)Y.sites, (void*)Y.packed);
      }
    }
    if (!L.exec || L.graph_key != key) {
      if (L.exec) (void)hipGraphExecDestroy(L.exec);
      if (L.graph) (void)hipGraphDestroy(L.graph);
      L.exec = nullptr;
      L.graph = nullptr;
      ICHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(stream);
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(stream, &gr);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        set_error("graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
        return ISING_ERR_DEVICE;
      }
      L.graph = gr;
      ICHK(hipGraphInstantiate(&L.exec, L.graph, nullptr, nullptr, 0));
      L.graph_key = key;
    }
    ICHK(hipGraphLaunch(L.exec, stream));
  } else {
    ICHK(enqueue(stream));
  }
  ICHK(hipEventRecord(L.ev1, stream));
  if (!L.done) ICHK(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
  ICHK(hipEventRecord(L.done, stream));
  L.done_recorded = true;
  return ISING_OK;
}

}  // namespace ising

using namespace ising;

const int32_t* fields_or_null(const ising_problem* p) { return p->g.fields ? p->dg.bf : nullptr; }

// Arguments of the per-pass kernels for a run of p in b.
PlainDev make_plain(const ising_problem* p, const RunBuffers& b, int R, uint64_t seed) {
  PlainDev P;
  memset(&P, 0, sizeof P);
  P.row = p->dg.row;
  P.adj = p->dg.adj;
  P.wgt = p->dg.wgt;
  P.grp = p->dg.grp;
  P.n_pad = p->g.n_pad;
  P.R = R;
  P.W = (int32_t)p->g.W;
  P.flags = (b.trace ? kJobTrace : 0);
  P.tq = b.tq;
  P.tq_off = b.tq_off;
  P.tq_len = b.tq_len;
  P.seed_lo = (uint32_t)seed;
  P.seed_hi = (uint32_t)(seed >> 32);
  P.init_spins = b.init_dev;
  P.spins = b.spins;
  P.field = b.field;
  P.best = static_cast<int8_t*>(b.best);
  P.energy = b.energy;
  P.eacc = b.eacc;
  P.best_cut = b.best_cut;
  P.best_sweep = b.best_sweep;
  P.snap = b.snap;
  P.accepts = b.accepts;
  P.trace = b.trace_buf;
  P.bfield = fields_or_null(p);
  return P;
}

// ================================================================ C ABI
extern "C" {

const char* ising_status_string(int status) {
  switch (status) {
    case ISING_OK: return "ok";
    case ISING_ERR_INVALID: return "invalid argument";
    case ISING_ERR_NOMEM: return "out of memory";
    case ISING_ERR_DEVICE: return "device error";
    case ISING_ERR_STATE: return "invalid state";
    case ISING_ERR_UNSUPPORTED: return "unsupported";
    case ISING_ERR_TIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

const char* ising_last_error(void) { return last_error(); }

int ising_set_allocator(ising_alloc_fn alloc, ising_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_error("give both an allocation and a free function, or neither");
    return ISING_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = alloc;
  g_free = free_fn;
  g_alloc_ctx = ctx;
  return ISING_OK;
}

int ising_create(int32_t n, int64_t m, const int32_t* u, const int32_t* v, const int32_t* w,
                 const int32_t* colour, ising_problem** out) {
  if (!out) return ISING_ERR_INVALID;
  TraceRange tr("ising_create");
  ising_problem* p = nullptr;
  try {
    p = new ising_problem();
  } catch (...) {
    return ISING_ERR_NOMEM;
  }
  int rc;
  try {
    rc = compile_graph(n, m, u, v, w, colour, p->g);
  } catch (...) {
    rc = ISING_ERR_NOMEM;
  }
  if (rc != ISING_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return ISING_OK;
}

int ising_destroy(ising_problem* p) {
  if (!p) return ISING_OK;
  if (p->run.valid && p->run.stream) (void)hipStreamSynchronize(p->run.stream);
  DeviceGuard g(p->dg.device);
  delete p;
  return ISING_OK;
}

int ising_problem_info(const ising_problem* p, ising_info* out) {
  if (!p || !out) return ISING_ERR_INVALID;
  ising_info i;
  i.n = p->g.n;
  i.n_colours = p->g.C;
  i.m = p->g.m;
  i.total_weight = p->g.W;
  i.kmax = p->g.kmax;
  i.max_degree = p->g.max_deg;
  i.unit_weights = p->g.unit ? 1 : 0;
  i.n_padded = p->g.n_pad;
  i.fields = p->g.fields ? 1 : 0;
  *out = i;
  return ISING_OK;
}

int ising_colouring(const ising_problem* p, int32_t* colour) {
  if (!p || !colour) return ISING_ERR_INVALID;
  memcpy(colour, p->g.colour.data(), sizeof(int32_t) * (size_t)p->g.n);
  return ISING_OK;
}

int ising_neighbour_labels(const ising_problem* p, int32_t* lab) {
  if (!p || !lab) return ISING_ERR_INVALID;
  if (p->g.lab4.empty()) {
    set_error("the problem has no degree-4 form");
    return ISING_ERR_UNSUPPORTED;
  }
  memcpy(lab, p->g.lab4.data(), sizeof(int32_t) * p->g.lab4.size());
  return ISING_OK;
}

int ising_eval_cut(const ising_problem* p, const int8_t* spins, int64_t* cut) {
  if (!p || !spins || !cut) return ISING_ERR_INVALID;
  int64_t c = 0;
  for (int64_t e = 0; e < p->g.m; ++e)
    if (spins[p->g.u[(size_t)e]] != spins[p->g.v[(size_t)e]]) c += p->g.w[(size_t)e];
  *cut = c;
  return ISING_OK;
}

int ising_set_fields(ising_problem* p, const int32_t* b) {
  if (!p) return ISING_ERR_INVALID;
  HostGraph& g = p->g;
  int64_t total = g.abs_total;
  if (b) {
    for (int32_t v = 0; v < g.n; ++v) {
      if (b[v] > 32768 || b[v] < -32768) {
        set_error("local field of vertex %d outside [-32768, 32768]", v);
        return ISING_ERR_INVALID;
      }
      total += 2 * (int64_t)std::abs(b[v]);
    }
    if (total >= ((int64_t)1 << 30)) {
      set_error("sum over vertices of sum |w| + 2 |b| must stay below 2^30");
      return ISING_ERR_INVALID;
    }
  }
  // the device copy may still be read by a run in flight
  if (p->run.valid && p->run.stream) (void)hipStreamSynchronize(p->run.stream);
  g.bpos.assign((size_t)g.n_pad, 0);
  g.fields = false;
  g.kmax = 0;
  for (int32_t v = 0; v < g.n; ++v) {
    const int32_t bv = b ? b[v] : 0;
    g.bpos[(size_t)g.pos[(size_t)v]] = bv;
    g.fields = g.fields || bv != 0;
    g.kmax = std::max<int32_t>(g.kmax, (int32_t)(g.wsum[(size_t)v] + 2 * (int64_t)std::abs(bv)));
  }
  // thresholds were built for the old kmax
  p->sched.table = Table();
  p->sched.kind = -1;
  p->temper.rows = Table();
  p->temper.betas.clear();
  if (p->dg.device >= 0) {
    DeviceGuard dg(p->dg.device);
    ICHK(hipMemcpy(p->dg.bf, g.bpos.data(), sizeof(int32_t) * (size_t)g.n_pad, hipMemcpyHostToDevice));
  }
  return ISING_OK;
}

int ising_threshold_table(const ising_schedule* s, int32_t kmax, uint64_t* out) {
  if (!s || kmax < 1 || !out) return ISING_ERR_INVALID;
  std::vector<double> beta;
  IRET(eval_schedule(s, beta));
  Table t;
  IRET(build_table(beta, kmax, t));
  for (int r = 0; r < t.S; ++r) {
    const int len = t.len[(size_t)r];
    for (int k = 1; k <= kmax; ++k) {
      uint64_t q;
      if (len == kAcceptAll) q = (uint64_t)1 << 32;
      else if (k <= len) q = (uint64_t)t.tq[(size_t)(t.off[(size_t)r] + k - 1)] + 1;
      else q = 0;
      out[(size_t)r * kmax + (k - 1)] = q;
    }
  }
  return ISING_OK;
}

int ising_set_initial_state(ising_problem* p, const int8_t* spins, int32_t n_replicas) {
  if (!p) return ISING_ERR_INVALID;
  if (!spins) {
    p->init.clear();
    p->init_R = 0;
    return ISING_OK;
  }
  if (n_replicas < 1) return ISING_ERR_INVALID;
  const size_t cnt = (size_t)n_replicas * (size_t)p->g.n;
  for (size_t i = 0; i < cnt; ++i)
    if (spins[i] != 1 && spins[i] != -1) {
      set_error("initial spins must be +-1");
      return ISING_ERR_INVALID;
    }
  p->init.assign(spins, spins + cnt);
  p->init_R = n_replicas;
  return ISING_OK;
}

int ising_set_trace(ising_problem* p, int32_t enable) {
  if (!p) return ISING_ERR_INVALID;
  p->trace = enable != 0;
  return ISING_OK;
}


// The table costs S * kmax exponentials, so it is kept while the schedule
// repeats.
extern "C++" int schedule_table(ising_problem* p, const ising_schedule* s) {
  auto& c = p->sched;
  const bool expl = s->kind == ISING_SCHED_EXPLICIT;
  if (c.table.id != 0 && c.kind == s->kind && c.n_sweeps == s->n_sweeps && s->n_sweeps > 0) {
    const bool same = expl ? (s->betas && c.betas.size() == (size_t)s->n_sweeps &&
                              memcmp(c.betas.data(), s->betas, sizeof(double) * c.betas.size()) == 0)
                           : (c.beta0 == s->beta0 && c.beta1 == s->beta1);
    if (same) return ISING_OK;
  }
  std::vector<double> beta;
  IRET(eval_schedule(s, beta));
  Table table;
  IRET(build_table(beta, p->g.kmax, table));
  c.table = std::move(table);
  c.kind = s->kind;
  c.n_sweeps = s->n_sweeps;
  c.beta0 = s->beta0;
  c.beta1 = s->beta1;
  c.betas.assign(expl ? s->betas : nullptr, expl ? s->betas + s->n_sweeps : nullptr);
  return ISING_OK;
}

int ising_anneal_range(ising_problem* p, const ising_schedule* s, int32_t n_replicas,
                       uint64_t seed, const ising_tuning* tuning, int32_t t_begin, int32_t t_end,
                       void* stream) {
  if (!p || !s || n_replicas < 1) return ISING_ERR_INVALID;
  TraceRange tr("ising_anneal_range");
  IRET(schedule_table(p, s));
  const Table& table = p->sched.table;
  if (t_begin < 0 || t_end <= t_begin || t_end > table.S) {
    set_error("sweep range [%d, %d) outside the schedule's %d sweeps", t_begin, t_end, table.S);
    return ISING_ERR_INVALID;
  }
  IRET(ensure_device(p));
  DeviceGuard dg(p->dg.device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  RunBuffers& b = p->run;
  PersistentConfig cfg;
  if (t_begin == 0) {
    IRET(resolve_config(p, table, n_replicas, tuning, cfg));
    IRET(prepare_run(p, table, n_replicas, cfg, st));
  } else {
    // a continuation: the same run, schedule and seed, at the sweep where
    // the last range stopped, in the launch configuration it used
    if (!b.valid || p->temper.valid || b.R != n_replicas || b.seed != seed ||
        b.t_done != t_begin || b.S != table.S || b.up_table != table.id || b.trace != p->trace) {
      set_error("no run of this schedule, seed and replica count stopped at sweep %d", t_begin);
      return ISING_ERR_STATE;
    }
    cfg = b.cfg;
    if (b.stream != st) ICHK(hipStreamSynchronize(b.stream));
    b.stream = st;
  }
  p->temper.valid = false;
  b.valid = false;
  if (cfg.path == ISING_PATH_PLAIN) {
    PlainDev P = make_plain(p, b, n_replicas, seed);
    static thread_local JobDev hjob;
    hjob = make_job(p->g, p->dg, b, n_replicas, seed, t_begin, t_end, cfg);
    ICHK(hipMemcpy(b.job_dev, &hjob, sizeof(JobDev), hipMemcpyHostToDevice));
    PlainPlan plan{table.S, p->g.C, p->g.cls.data()};
    plan.t_begin = t_begin;
    plan.t_end = t_end;
    ICHK(hipEventRecord(b.ev0, st));
    ICHK(launch_plain_anneal(P, plan, st));
    ICHK(launch_argmax(b.job_dev, 1, st));
    ICHK(hipEventRecord(b.ev1, st));
  } else {
    std::vector<JobSpec> js{JobSpec{&p->g, &p->dg, &b, n_replicas, seed, t_begin, t_end}};
    ICHK(hipEventRecord(b.ev0, st));
    IRET(run_persistent(p->launcher, js, cfg, st, st != nullptr));
    ICHK(hipEventRecord(b.ev1, st));
  }
  b.cfg = cfg;
  b.seed = seed;
  b.t_done = t_end;
  b.valid = true;
  return ISING_OK;
}

int ising_anneal_tuned(ising_problem* p, const ising_schedule* s, int32_t n_replicas,
                       uint64_t seed, const ising_tuning* tuning, void* stream) {
  if (!p || !s || s->n_sweeps < 1) return ISING_ERR_INVALID;
  return ising_anneal_range(p, s, n_replicas, seed, tuning, 0, s->n_sweeps, stream);
}

// ---------------------------------------------------------------- checkpoint
namespace {
struct CheckpointHeader {
  uint64_t magic;
  int32_t version, R, S, path, G, block, adj, t_done, n_pad, trace, init;
  uint64_t seed, arena_used, table_hash;
};
constexpr uint64_t kCheckpointMagic = 0x31544B4347534949ull;  // "IISGCKT1"

uint64_t table_hash(const Table& t) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the rows
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  };
  mix(t.tq.data(), sizeof(uint32_t) * t.tq.size());
  mix(t.off.data(), sizeof(int32_t) * t.off.size());
  mix(t.len.data(), sizeof(int32_t) * t.len.size());
  mix(&t.kmax, sizeof t.kmax);
  return h;
}
}  // namespace

int ising_checkpoint_size(const ising_problem* p, uint64_t* bytes) {
  if (!p || !bytes) return ISING_ERR_INVALID;
  if (!p->run.valid || p->temper.valid) {
    set_error("no anneal to checkpoint");
    return ISING_ERR_STATE;
  }
  *bytes = sizeof(CheckpointHeader) + p->run.arena.used;
  return ISING_OK;
}

int ising_checkpoint_save(ising_problem* p, void* buf) {
  uint64_t bytes = 0;
  if (!buf) return ISING_ERR_INVALID;
  IRET(ising_checkpoint_size(p, &bytes));
  RunBuffers& b = p->run;
  DeviceGuard g(p->dg.device);
  ICHK(hipStreamSynchronize(b.stream));
  CheckpointHeader h;
  memset(&h, 0, sizeof h);
  h.magic = kCheckpointMagic;
  h.version = 1;
  h.R = b.R;
  h.S = b.S;
  h.path = b.cfg.path;
  h.G = b.cfg.G;
  h.block = b.cfg.block;
  h.adj = b.cfg.adj;
  h.t_done = b.t_done;
  h.n_pad = p->g.n_pad;
  h.trace = b.trace ? 1 : 0;
  h.init = b.init_dev ? 1 : 0;
  h.seed = b.seed;
  h.arena_used = b.arena.used;
  h.table_hash = table_hash(b.table);
  memcpy(buf, &h, sizeof h);
  ICHK(hipMemcpy(static_cast<char*>(buf) + sizeof h, b.arena.base, b.arena.used, hipMemcpyDeviceToHost));
  return ISING_OK;
}

int ising_checkpoint_load(ising_problem* p, const ising_schedule* s, const void* buf,
                          uint64_t bytes, void* stream) {
  if (!p || !s || !buf || bytes < sizeof(CheckpointHeader)) return ISING_ERR_INVALID;
  CheckpointHeader h;
  memcpy(&h, buf, sizeof h);
  if (h.magic != kCheckpointMagic || h.version != 1 || bytes != sizeof h + h.arena_used ||
      h.n_pad != p->g.n_pad) {
    set_error("not a checkpoint of this problem");
    return ISING_ERR_INVALID;
  }
  IRET(schedule_table(p, s));
  const Table& table = p->sched.table;
  if (table.S != h.S || table_hash(table) != h.table_hash) {
    set_error("the checkpoint was taken under another schedule");
    return ISING_ERR_INVALID;
  }
  if ((p->trace ? 1 : 0) != h.trace || (p->init_R > 0 ? 1 : 0) != h.init) {
    set_error("tracing and given initial states must be as when the checkpoint was taken");
    return ISING_ERR_STATE;
  }
  IRET(ensure_device(p));
  DeviceGuard dg(p->dg.device);
  PersistentConfig cfg;
  cfg.path = h.path;
  cfg.G = h.G;
  cfg.block = h.block;
  cfg.adj = h.adj;
  IRET(check_config(p->g, table, h.R, cfg));
  hipStream_t st = static_cast<hipStream_t>(stream);
  IRET(prepare_run(p, table, h.R, cfg, st));
  RunBuffers& b = p->run;
  if (b.arena.used != h.arena_used) {
    set_error("the checkpoint was written by a library with another buffer layout");
    return ISING_ERR_INVALID;
  }
  // the uploads of prepare_run go first, then the saved bytes over them
  ICHK(hipStreamSynchronize(st));
  ICHK(hipMemcpy(b.arena.base, static_cast<const char*>(buf) + sizeof h, h.arena_used,
                 hipMemcpyHostToDevice));
  // the saved bytes include the same tables, but force a fresh upload
  // should the next run bring another schedule
  b.cfg = cfg;
  b.seed = h.seed;
  b.t_done = h.t_done;
  b.valid = true;
  p->temper.valid = false;
  return ISING_OK;
}

int ising_anneal(ising_problem* p, const ising_schedule* s, int32_t n_replicas, uint64_t seed,
                 void* stream) {
  return ising_anneal_tuned(p, s, n_replicas, seed, nullptr, stream);
}

static int sync_results(ising_problem* p) {
  if (!p) return ISING_ERR_INVALID;
  if (!p->run.valid) {
    set_error("no anneal has run on this problem");
    return ISING_ERR_STATE;
  }
  DeviceGuard g(p->dg.device);
  ICHK(hipStreamSynchronize(p->run.stream));
  return ISING_OK;
}

int ising_cut(ising_problem* p, int64_t* best_cut, int32_t* best_replica, int64_t* per_replica) {
  IRET(sync_results(p));
  DeviceGuard g(p->dg.device);
  RunBuffers& b = p->run;
  unsigned long long key = 0;
  ICHK(hipMemcpy(&key, b.argmax, sizeof key, hipMemcpyDeviceToHost));
  if (per_replica) {
    std::vector<int32_t> tmp((size_t)b.R);
    ICHK(hipMemcpy(tmp.data(), b.best_cut, sizeof(int32_t) * b.R, hipMemcpyDeviceToHost));
    for (int r = 0; r < b.R; ++r) per_replica[r] = tmp[(size_t)r];
  }
  const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
  if (best_cut) *best_cut = (int64_t)(int32_t)(hi ^ 0x80000000u);
  if (best_replica) *best_replica = (int32_t)(0xFFFFFFFFu - lo);
  return ISING_OK;
}

static int gather_state(ising_problem* p, const void* buf, int layout, int r,
                        std::vector<int32_t>& out) {
  RunBuffers& b = p->run;
  out.assign((size_t)p->g.n, 0);
  ICHK(launch_gather(buf, layout, b.R, p->g.n_pad, r, p->dg.pos, p->g.n, b.gather, b.stream));
  ICHK(hipStreamSynchronize(b.stream));
  ICHK(hipMemcpy(out.data(), b.gather, sizeof(int32_t) * (size_t)p->g.n, hipMemcpyDeviceToHost));
  return ISING_OK;
}

int ising_best_state(ising_problem* p, int8_t* spins) {
  if (!spins) return ISING_ERR_INVALID;
  int32_t r = 0;
  IRET(ising_cut(p, nullptr, &r, nullptr));
  DeviceGuard g(p->dg.device);
  std::vector<int32_t> tmp;
  IRET(gather_state(p, p->run.best, p->run.layout_best, r, tmp));
  for (int32_t v = 0; v < p->g.n; ++v) spins[v] = (int8_t)tmp[(size_t)v];
  return ISING_OK;
}

int ising_replica_results(ising_problem* p, int32_t* best_sweep, int64_t* accepts,
                          int64_t* final_energy) {
  IRET(sync_results(p));
  DeviceGuard g(p->dg.device);
  RunBuffers& b = p->run;
  if (best_sweep)
    ICHK(hipMemcpy(best_sweep, b.best_sweep, sizeof(int32_t) * b.R, hipMemcpyDeviceToHost));
  if (accepts) {
    std::vector<unsigned long long> tmp((size_t)b.R);
    ICHK(hipMemcpy(tmp.data(), b.accepts, sizeof(unsigned long long) * b.R, hipMemcpyDeviceToHost));
    for (int r = 0; r < b.R; ++r) accepts[r] = (int64_t)tmp[(size_t)r];
  }
  if (final_energy) {
    std::vector<int32_t> tmp((size_t)b.R);
    ICHK(hipMemcpy(tmp.data(), b.energy, sizeof(int32_t) * b.R, hipMemcpyDeviceToHost));
    for (int r = 0; r < b.R; ++r) final_energy[r] = tmp[(size_t)r];
  }
  return ISING_OK;
}

int ising_replica_state(ising_problem* p, int32_t r, int8_t* best_spins, int8_t* final_spins) {
  IRET(sync_results(p));
  if (r < 0 || r >= p->run.R) return ISING_ERR_INVALID;
  DeviceGuard g(p->dg.device);
  RunBuffers& b = p->run;
  std::vector<int32_t> tmp;
  if (best_spins) {
    IRET(gather_state(p, b.best, b.layout_best, r, tmp));
    for (int32_t v = 0; v < p->g.n; ++v) best_spins[v] = (int8_t)tmp[(size_t)v];
  }
  if (final_spins) {
    const void* src = b.path == ISING_PATH_PLAIN ? (const void*)b.spins : (const void*)b.save;
    IRET(gather_state(p, src, b.layout_final, r, tmp));
    for (int32_t v = 0; v < p->g.n; ++v) final_spins[v] = (int8_t)tmp[(size_t)v];
  }
  return ISING_OK;
}

int ising_replica_field(ising_problem* p, int32_t r, int32_t* field) {
  IRET(sync_results(p));
  if (r < 0 || r >= p->run.R || !field) return ISING_ERR_INVALID;
  RunBuffers& b = p->run;
  if (b.layout_field < 0) {
    set_error("the multispin path keeps no field array");
    return ISING_ERR_UNSUPPORTED;
  }
  DeviceGuard g(p->dg.device);
  std::vector<int32_t> tmp;
  const void* src = b.path == ISING_PATH_PLAIN ? (const void*)b.field : (const void*)b.save;
  IRET(gather_state(p, src, b.layout_field, r, tmp));
  memcpy(field, tmp.data(), sizeof(int32_t) * (size_t)p->g.n);
  return ISING_OK;
}

int ising_energy_trace(ising_problem* p, int64_t* out) {
  IRET(sync_results(p));
  if (!out) return ISING_ERR_INVALID;
  RunBuffers& b = p->run;
  if (!b.trace_buf) {
    set_error("tracing was not enabled for the last anneal");
    return ISING_ERR_STATE;
  }
  DeviceGuard g(p->dg.device);
  std::vector<int32_t> tmp((size_t)b.S * b.R);
  ICHK(hipMemcpy(tmp.data(), b.trace_buf, sizeof(int32_t) * tmp.size(), hipMemcpyDeviceToHost));
  for (int r = 0; r < b.R; ++r)
    for (int t = 0; t < b.S; ++t) out[(size_t)r * b.S + t] = tmp[(size_t)t * b.R + r];
  return ISING_OK;
}

int ising_last_run_info(const ising_problem* p, int32_t* n_replicas, int32_t* n_sweeps,
                        int32_t* path) {
  if (!p) return ISING_ERR_INVALID;
  if (!p->run.valid) {
    set_error("no anneal has run on this problem");
    return ISING_ERR_STATE;
  }
  if (n_replicas) *n_replicas = p->run.R;
  if (n_sweeps) *n_sweeps = p->run.S;
  if (path) *path = p->run.path;
  return ISING_OK;
}

int ising_last_anneal_ms(ising_problem* p, double* ms) {
  IRET(sync_results(p));
  if (!ms) return ISING_ERR_INVALID;
  float f = 0;
  ICHK(hipEventElapsedTime(&f, p->run.ev0, p->run.ev1));
  *ms = f;
  return ISING_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- config
int tune_lookup(const ising::HostGraph& g, const ising::Table& t, int R, ising::PersistentConfig& c);

int resolve_config(ising_problem* p, const Table& table, int R, const ising_tuning* t,
                   PersistentConfig& cfg) {
  const int path = t ? t->path : ISING_PATH_AUTO;
  if (path == ISING_PATH_AUTO) {
    if (tune_lookup(p->g, table, R, cfg) != ISING_OK) cfg = heuristic_config(p->g, table, R);
    return ISING_OK;
  }
  cfg.path = path;
  cfg.G = t->replicas_per_block > 0 ? t->replicas_per_block : 1;
  cfg.block = t->block_threads > 0 ? t->block_threads : (path == ISING_PATH_MSC ? 256 : 1024);
  cfg.adj = t->lds_adjacency;
  if (path == ISING_PATH_PLAIN) {
    cfg.G = 1;
    cfg.block = 256;
  }
  return check_config(p->g, table, R, cfg);
}
