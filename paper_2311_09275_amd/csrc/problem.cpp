// problem.cpp -- problem compiler, schedules and acceptance thresholds.
//
// Problem (paper Sec. II.A): weighted MaxCut on n vertices, couplings
// J = -w.  The compiled form is colour-major: colour classes in order, each
// class's vertices in ascending id, each class padded to a multiple of four
// positions so that aligned quadruples are the random-number groups.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <atomic>

#include "runtime.h"

namespace ising {

namespace {
thread_local char g_err[512];
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}
const char* last_error() { return g_err; }

// ---------------------------------------------------------------- graph
// Neighbour labels of a 4-regular graph (CSR deg/nb in vertex ids) such
// that lab[4 v + e] = u implies lab[4 u + (e ^ 1)] = v: an edge carries
// labels 2f and 2f + 1 at its two ends.  Closed walks over unused edges
// orient every edge with two out- and two in-edges per vertex (all degrees
// are even, so a walk can only stop where it started).  The graph that
// joins each vertex's out side to the in side of its out-neighbours is
// then 2-regular and bipartite, a union of even cycles; taking their edges
// alternately gives two perfect matchings f = 0, 1, and an edge v -> u of
// matching f is labelled 2f at v and 2f + 1 at u.  False if a check fails.
// First choice: the caller's edge order, when it already is such a
// labelling -- edge e oriented u[e] -> v[e], in matching f = the rank of e
// among u[e]'s edges of that orientation.  A torus listed as (v, right),
// (v, down) gives the same labels to the same directions everywhere
// (right, left, down, up), so the pushes of one instruction land on
// neighbours at one offset, in distinct LDS banks.
static bool edge_order_labels(int32_t n, int64_t m, const int32_t* u, const int32_t* v,
                              std::vector<int32_t>& lab) {
  std::vector<int> n_out((size_t)n, 0), n_in((size_t)n, 0);
  lab.assign((size_t)4 * n, -1);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t a = u[e], b = v[e];
    const int f = n_out[(size_t)a]++;
    if (f > 1 || n_in[(size_t)b]++ > 1) return false;
    if (lab[4 * (size_t)b + 2 * f + 1] >= 0) return false;  // two in-edges of one matching
    lab[4 * (size_t)a + 2 * f] = b;
    lab[4 * (size_t)b + 2 * f + 1] = a;
  }
  for (int32_t a = 0; a < n; ++a)
    for (int e = 0; e < 4; ++e) {
      const int32_t b = lab[4 * (size_t)a + e];
      if (b < 0 || lab[4 * (size_t)b + (e ^ 1)] != a) return false;
    }
  return true;
}

static bool bond_labels(int32_t n, const std::vector<int32_t>& deg, const std::vector<int32_t>& nb,
                        std::vector<int32_t>& lab) {
  const size_t H = (size_t)deg[(size_t)n];  // half-edges
  std::vector<int32_t> mate(H, -1), head(H, 0);
  for (int32_t v = 0; v < n; ++v)
    for (int32_t a = deg[(size_t)v]; a < deg[(size_t)v + 1]; ++a) {
      head[(size_t)a] = v;
      const int32_t u = nb[(size_t)a];
      for (int32_t b = deg[(size_t)u]; b < deg[(size_t)u + 1]; ++b)
        if (nb[(size_t)b] == v) mate[(size_t)a] = b;
      if (mate[(size_t)a] < 0) return false;
    }
  // orientation: dir[a] = 1 when half-edge a (head[a] -> nb[a]) was walked
  std::vector<uint8_t> used(H, 0), dir(H, 0);
  std::vector<int32_t> next(deg.begin(), deg.end() - 1);
  for (int32_t s0 = 0; s0 < n; ++s0) {
    for (;;) {
      int32_t v = s0;
      bool moved = false;
      for (;;) {
        while (next[(size_t)v] < deg[(size_t)v + 1] && used[(size_t)next[(size_t)v]]) ++next[(size_t)v];
        if (next[(size_t)v] == deg[(size_t)v + 1]) break;
        const int32_t a = next[(size_t)v];
        used[(size_t)a] = used[(size_t)mate[(size_t)a]] = 1;
        dir[(size_t)a] = 1;
        v = nb[(size_t)a];
        moved = true;
      }
      if (!moved) break;
      if (v != s0) return false;
    }
  }
  // out- and in-half-edges per vertex (walked half-edges leave head[a])
  std::vector<int32_t> outs((size_t)2 * n, -1), ins((size_t)2 * n, -1);
  std::vector<int> n_out((size_t)n, 0), n_in((size_t)n, 0);
  for (size_t a = 0; a < H; ++a) {
    if (!dir[a]) continue;
    const int32_t v = head[a], u = nb[a];
    if (n_out[(size_t)v] > 1 || n_in[(size_t)u] > 1) return false;
    outs[2 * (size_t)v + (size_t)n_out[(size_t)v]++] = (int32_t)a;
    ins[2 * (size_t)u + (size_t)n_in[(size_t)u]++] = (int32_t)a;
  }
  for (int32_t v = 0; v < n; ++v)
    if (n_out[(size_t)v] != 2 || n_in[(size_t)v] != 2) return false;
  // alternate the edges of each out/in cycle between matchings 0 and 1
  std::vector<int8_t> fac(H, -1);
  for (size_t a0 = 0; a0 < H; ++a0) {
    if (!dir[a0] || fac[a0] >= 0) continue;
    int32_t a = (int32_t)a0;
    int f = 0;
    while (fac[(size_t)a] < 0) {
      fac[(size_t)a] = (int8_t)f;
      // the other in-edge of a's target, then the other out-edge of its tail
      const int32_t u = nb[(size_t)a];
      const int32_t b = ins[2 * (size_t)u] == a ? ins[2 * (size_t)u + 1] : ins[2 * (size_t)u];
      if (fac[(size_t)b] >= 0) {
        if (fac[(size_t)b] == f) return false;
        break;
      }
      fac[(size_t)b] = (int8_t)(1 - f);
      const int32_t t = head[(size_t)b];
      a = outs[2 * (size_t)t] == b ? outs[2 * (size_t)t + 1] : outs[2 * (size_t)t];
      if (fac[(size_t)a] >= 0 && fac[(size_t)a] != f) return false;
    }
  }
  lab.assign((size_t)4 * n, -1);
  for (size_t a = 0; a < H; ++a) {
    if (!dir[a]) continue;
    const int32_t v = head[a], u = nb[a], f = fac[a];
    if (f < 0 || lab[4 * (size_t)v + 2 * f] >= 0 || lab[4 * (size_t)u + 2 * f + 1] >= 0) return false;
    lab[4 * (size_t)v + 2 * f] = u;
    lab[4 * (size_t)u + 2 * f + 1] = v;
  }
  for (int32_t v = 0; v < n; ++v)
    for (int e = 0; e < 4; ++e) {
      const int32_t u = lab[4 * (size_t)v + e];
      if (u < 0 || lab[4 * (size_t)u + (e ^ 1)] != v) return false;
    }
  return true;
}

int compile_graph(int32_t n, int64_t m, const int32_t* u, const int32_t* v, const int32_t* w,
                  const int32_t* colour, HostGraph& g) {
  if (n < 1 || n >= (1 << 28) || m < 0) {
    set_error("n must be in [1, 2^28) and m >= 0");
    return ISING_ERR_INVALID;
  }
  if (m > 0 && (!u || !v || !w)) {
    set_error("edge arrays are NULL");
    return ISING_ERR_INVALID;
  }
  if (m > (int64_t)1 << 30) {
    set_error("too many edges");
    return ISING_ERR_INVALID;
  }
  g = HostGraph();
  g.n = n;
  g.m = m;
  g.u.assign(u, u + m);
  g.v.assign(v, v + m);
  g.w.assign(w, w + m);
  int64_t abs_total = 0;
  std::vector<uint64_t> keys((size_t)m);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t a = u[e], b = v[e], we = w[e];
    if (a < 0 || b < 0 || a >= n || b >= n) {
      set_error("edge %lld: vertex id out of range", (long long)e);
      return ISING_ERR_INVALID;
    }
    if (a == b) {
      set_error("edge %lld: self loop", (long long)e);
      return ISING_ERR_INVALID;
    }
    if (we == 0 || we > 32768 || we < -32768) {
      set_error("edge %lld: weight must be nonzero with |w| <= 32768", (long long)e);
      return ISING_ERR_INVALID;
    }
    abs_total += 2 * (int64_t)(we < 0 ? -we : we);
    keys[(size_t)e] = ((uint64_t)(uint32_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
  }
  if (abs_total >= ((int64_t)1 << 30)) {
    set_error("sum of |w| over vertex neighbourhoods must stay below 2^30");
    return ISING_ERR_INVALID;
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end()) {
    set_error("repeated undirected edge");
    return ISING_ERR_INVALID;
  }

  // adjacency in original ids
  std::vector<int32_t> deg((size_t)n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    ++deg[(size_t)u[e] + 1];
    ++deg[(size_t)v[e] + 1];
  }
  for (int32_t i = 0; i < n; ++i) deg[(size_t)i + 1] += deg[(size_t)i];
  std::vector<int32_t> nb((size_t)(2 * m)), nw((size_t)(2 * m)), fill(deg.begin(), deg.end() - 1);
  for (int64_t e = 0; e < m; ++e) {
    nb[(size_t)fill[(size_t)u[e]]] = v[e];
    nw[(size_t)fill[(size_t)u[e]]++] = w[e];
    nb[(size_t)fill[(size_t)v[e]]] = u[e];
    nw[(size_t)fill[(size_t)v[e]]++] = w[e];
  }
  g.W = 0;
  for (int64_t e = 0; e < m; ++e) g.W += w[e];
  g.kmax = 0;
  g.max_deg = 0;
  g.unit = true;
  g.wsum.assign((size_t)n, 0);
  g.abs_total = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t s = 0;
    for (int32_t a = deg[(size_t)i]; a < deg[(size_t)i + 1]; ++a) {
      s += std::abs(nw[(size_t)a]);
      if (std::abs(nw[(size_t)a]) != 1) g.unit = false;
    }
    g.wsum[(size_t)i] = s;
    g.abs_total += s;
    g.kmax = std::max<int32_t>(g.kmax, (int32_t)s);
    g.max_deg = std::max<int32_t>(g.max_deg, deg[(size_t)i + 1] - deg[(size_t)i]);
  }

  // colouring: supplied (checked proper) or greedy first fit in id order
  g.colour.assign((size_t)n, 0);
  if (colour) {
    for (int32_t i = 0; i < n; ++i) {
      if (colour[i] < 0 || colour[i] >= 1024) {
        set_error("colour of vertex %d out of [0, 1024)", i);
        return ISING_ERR_INVALID;
      }
      g.colour[(size_t)i] = colour[i];
    }
    for (int64_t e = 0; e < m; ++e)
      if (colour[u[e]] == colour[v[e]]) {
        set_error("colouring is not proper at edge %lld", (long long)e);
        return ISING_ERR_INVALID;
      }
  } else {
    std::vector<int32_t> mark((size_t)n + 2, -1);
    for (int32_t i = 0; i < n; ++i) {
      for (int32_t a = deg[(size_t)i]; a < deg[(size_t)i + 1]; ++a)
        if (nb[(size_t)a] < i) mark[(size_t)g.colour[(size_t)nb[(size_t)a]]] = i;
      int32_t c = 0;
      while (mark[(size_t)c] == i) ++c;
      g.colour[(size_t)i] = c;
    }
  }
  g.C = 0;
  for (int32_t i = 0; i < n; ++i) g.C = std::max(g.C, g.colour[(size_t)i] + 1);

  // colour-major positions, classes padded to multiples of four
  std::vector<int32_t> class_size((size_t)g.C, 0);
  for (int32_t i = 0; i < n; ++i) ++class_size[(size_t)g.colour[(size_t)i]];
  std::vector<int32_t> class_start((size_t)g.C + 1, 0);
  for (int32_t c = 0; c < g.C; ++c)
    class_start[(size_t)c + 1] = class_start[(size_t)c] + ((class_size[(size_t)c] + 3) & ~3);
  g.n_pad = class_start[(size_t)g.C];
  if ((int64_t)g.n_pad >= ((int64_t)1 << 28)) {
    set_error("too many vertices after padding");
    return ISING_ERR_INVALID;
  }
  g.pos.assign((size_t)n, 0);
  g.orig.assign((size_t)g.n_pad, -1);
  std::vector<int32_t> cur(class_start.begin(), class_start.end() - 1);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t p = cur[(size_t)g.colour[(size_t)i]]++;
    g.pos[(size_t)i] = p;
    g.orig[(size_t)p] = i;
  }
  g.grp.assign((size_t)g.n_pad / 4, 0);
  for (int32_t q = 0; q < g.n_pad / 4; ++q) {
    int cnt = 0;
    for (int j = 0; j < 4; ++j) cnt += g.orig[(size_t)(4 * q + j)] >= 0;
    // padding only at class ends, so a group's first slot is always real
    g.grp[(size_t)q] = g.orig[(size_t)(4 * q)] | ((cnt - 1) << kGroupCountShift);
  }
  g.cls.assign((size_t)(2 * g.C), 0);
  for (int32_t c = 0; c < g.C; ++c) {
    g.cls[(size_t)(2 * c)] = class_start[(size_t)c] / 4;
    g.cls[(size_t)(2 * c + 1)] = class_start[(size_t)c + 1] / 4;
  }
  g.row.assign((size_t)g.n_pad + 1, 0);
  for (int32_t p = 0; p < g.n_pad; ++p) {
    const int32_t i = g.orig[(size_t)p];
    g.row[(size_t)p + 1] = g.row[(size_t)p] + (i >= 0 ? deg[(size_t)i + 1] - deg[(size_t)i] : 0);
  }
  g.adj.assign((size_t)(2 * m), 0);
  g.wgt.assign((size_t)(2 * m), 0);
  g.adjm.assign((size_t)(2 * m), 0);
  for (int32_t p = 0; p < g.n_pad; ++p) {
    const int32_t i = g.orig[(size_t)p];
    if (i < 0) continue;
    int32_t o = g.row[(size_t)p];
    for (int32_t a = deg[(size_t)i]; a < deg[(size_t)i + 1]; ++a, ++o) {
      const int32_t q = g.pos[(size_t)nb[(size_t)a]];
      g.adj[(size_t)o] = q;
      g.wgt[(size_t)o] = nw[(size_t)a];
      g.adjm[(size_t)o] = ((uint32_t)q << 1) | (nw[(size_t)a] > 0 ? 1u : 0u);
    }
  }
  g.aw.assign((size_t)(4 * m), 0);
  for (size_t a = 0; a < (size_t)(2 * m); ++a) {
    g.aw[2 * a] = g.adj[a];
    g.aw[2 * a + 1] = g.wgt[a];
  }
  g.gbase.assign((size_t)g.n_pad / 4, 0);
  g.gdeg.assign((size_t)g.n_pad / 4, 0);
  for (int32_t q = 0; q < g.n_pad / 4; ++q) {
    g.gbase[(size_t)q] = g.row[(size_t)(4 * q)];
    uint32_t packed = 0;
    for (int j = 0; j < 4; ++j) {
      const int32_t d = g.row[(size_t)(4 * q + j + 1)] - g.row[(size_t)(4 * q + j)];
      packed |= (uint32_t)std::min(d, 255) << (8 * j);
    }
    g.gdeg[(size_t)q] = packed;
  }
  g.deg4 = n > 0;
  for (int32_t i = 0; i < n && g.deg4; ++i) g.deg4 = deg[(size_t)i + 1] - deg[(size_t)i] == 4;
  std::vector<int32_t> lab;
  if (g.deg4 && g.unit && field_state_words(g.n_pad) <= (1 << 16) &&
      (edge_order_labels(n, m, u, v, lab) || bond_labels(n, deg, nb, lab))) {
    g.lab4 = lab;
    const size_t ng = (size_t)g.n_pad / 4;
    g.adj4.assign((size_t)kDeg4BlockWords * ng, 0u);
    for (size_t q = 0; q < ng; ++q) {
      uint32_t* blk = g.adj4.data() + (size_t)kDeg4BlockWords * q;
      blk[8] = (uint32_t)(g.grp[q] & kGroupLeaderMask);
      for (int j = 0; j < 4; ++j) {
        const int32_t i = g.orig[4 * q + (size_t)j];
        if (i < 0) continue;  // padding slot: never pushed
        for (int e = 0; e < 4; ++e) {
          // neighbours in label order, as words of the FIELD kernel's
          // tiled state (tile_word), and the sign of each weight
          const int32_t nbr = lab[4 * (size_t)i + e];
          const uint32_t pos = (uint32_t)g.pos[(size_t)nbr];
          const uint32_t word = (uint32_t)tile_word((int)(pos >> 2), (int)(pos & 3u));
          blk[2 * j + e / 2] |= word << (16 * (e & 1));
          int32_t we = 0;
          for (int32_t a = deg[(size_t)i]; a < deg[(size_t)i + 1]; ++a)
            if (nb[(size_t)a] == nbr) we = nw[(size_t)a];
          if (we > 0) blk[9] |= 1u << (4 * j + e);
        }
      }
    }
    // The multispin degree-4 form keeps every state element next to its
    // complement (element 2 i + 1 = NOT element 2 i), so that an entry can
    // name the copy that already carries its edge's sign: entry (j, e) is
    // 2 tile_word(neighbour) + (w > 0), and the element read there XOR the
    // vertex's own element is the bond's "unsatisfied" mask (w s_v s_u = +1).
    if (2 * field_state_words(g.n_pad) <= (1 << 16)) {
      g.adj4m.assign((size_t)kDeg4MscBlockWords * ng, 0u);
      for (size_t q = 0; q < ng; ++q) {
        uint32_t* blk = g.adj4m.data() + (size_t)kDeg4MscBlockWords * q;
        for (int j = 0; j < 4; ++j) {
          const int32_t i = g.orig[4 * q + (size_t)j];
          if (i < 0) continue;  // padding slot: its flips are masked off
          for (int e = 0; e < 4; ++e) {
            const int32_t nbr = lab[4 * (size_t)i + e];
            const uint32_t pos = (uint32_t)g.pos[(size_t)nbr];
            int32_t we = 0;
            for (int32_t a = deg[(size_t)i]; a < deg[(size_t)i + 1]; ++a)
              if (nb[(size_t)a] == nbr) we = nw[(size_t)a];
            const uint32_t ent = 2u * (uint32_t)tile_word((int)(pos >> 2), (int)(pos & 3u)) +
                                 (we > 0 ? 1u : 0u);
            blk[2 * j + e / 2] |= ent << (16 * (e & 1));
          }
        }
      }
    }
  }
  g.fields = false;
  g.bpos.assign((size_t)g.n_pad, 0);
  return ISING_OK;
}

// ---------------------------------------------------------------- schedule
int eval_schedule(const ising_schedule* s, std::vector<double>& beta) {
  if (!s || s->n_sweeps <= 0) {
    set_error("schedule needs n_sweeps >= 1");
    return ISING_ERR_INVALID;
  }
  const int S = s->n_sweeps;
  beta.assign((size_t)S, 0.0);
  if (s->kind == ISING_SCHED_EXPLICIT) {
    if (!s->betas) {
      set_error("explicit schedule without betas");
      return ISING_ERR_INVALID;
    }
    for (int t = 0; t < S; ++t) beta[(size_t)t] = s->betas[t];
  } else if (s->kind == ISING_SCHED_LINEAR || s->kind == ISING_SCHED_GEOMETRIC) {
    const double b0 = s->beta0, b1 = s->beta1;
    if (!std::isfinite(b0) || !std::isfinite(b1) || b0 < 0 || b1 < 0) {
      set_error("beta0 and beta1 must be finite and >= 0");
      return ISING_ERR_INVALID;
    }
    if (s->kind == ISING_SCHED_GEOMETRIC && (b0 <= 0 || b1 <= 0)) {
      set_error("a geometric schedule needs beta0, beta1 > 0");
      return ISING_ERR_INVALID;
    }
    for (int t = 0; t < S; ++t) {
      if (S == 1) {
        beta[(size_t)t] = b0;
        continue;
      }
      const double frac = (double)t / (double)(S - 1);
      beta[(size_t)t] = s->kind == ISING_SCHED_LINEAR ? b0 + (b1 - b0) * frac
                                                      : b0 * std::pow(b1 / b0, frac);
    }
  } else {
    set_error("unknown schedule kind %d", s->kind);
    return ISING_ERR_INVALID;
  }
  for (int t = 0; t < S; ++t)
    if (!std::isfinite(beta[(size_t)t]) || beta[(size_t)t] < 0) {
      set_error("beta_%d is not finite and >= 0", t);
      return ISING_ERR_INVALID;
    }
  return ISING_OK;
}

// Metropolis acceptance exp(-beta dE), dE = 2k, quantised to 32 bits:
// a move with k > 0 is accepted iff a uniform u32 draw is below Tq.
uint64_t threshold_q32(double beta, int64_t k) {
  double x = -2.0 * (double)k;
  x = x * beta;
  const double a = std::exp(x);
  if (a >= 1.0) return (uint64_t)1 << 32;
  return (uint64_t)std::floor(std::ldexp(a, 32));
}

// Rows hold Tq - 1 for k = 1 .. len_t, where len_t is the last k with
// Tq >= 1 (Tq falls with k); beta = 0 rows are marked accept-all.
int build_table(const std::vector<double>& beta, int32_t kmax, Table& t) {
  static std::atomic<uint64_t> next_id{1};
  t = Table();
  t.id = next_id.fetch_add(1);
  t.S = (int)beta.size();
  t.kmax = kmax;
  t.off.assign((size_t)t.S, 0);
  t.len.assign((size_t)t.S, 0);
  for (int s = 0; s < t.S; ++s) {
    t.off[(size_t)s] = (int32_t)t.tq.size();
    if (beta[(size_t)s] == 0.0) {
      t.len[(size_t)s] = kAcceptAll;
      continue;
    }
    int32_t len = 0;
    for (int64_t k = 1; k <= kmax; ++k) {
      const uint64_t q = threshold_q32(beta[(size_t)s], k);
      if (q == 0) break;
      if ((int64_t)t.tq.size() >= kMaxTableEntries) {
        set_error("threshold table exceeds 2^26 entries");
        return ISING_ERR_INVALID;
      }
      t.tq.push_back((uint32_t)(q - 1));
      ++len;
    }
    t.len[(size_t)s] = len;
    t.kw = std::max(t.kw, len);
  }
  if (t.tq.empty()) t.tq.push_back(0);
  return ISING_OK;
}

}  // namespace ising
