// Geometric modified nested dissection with interfaces on a box grid
// (Section 2.3, Figs. mnd and mnd_multilvl; geometric partitioning of the
// graph of A^T A for grid problems, Section 4).
//
// Separators are two grid layers thick so that they cut the graph of A^T A
// (which couples points up to two steps apart).  A box [lo, hi) splits on its
// longest axis (lowest axis on ties) at m = lo + floor((w-2)/2): separator
// {m, m+1}, low child [lo, m), high child [m+2, hi).  Nodes are heap-numbered
// (root 1, children 2k, 2k+1); level = bit length, leaves at level L.
//
// A separator point of node B is pushed onto the adjacent layer of each child
// (m-1 low, m+2 high) and descended to the deepest node containing it:
// (dl, dh).  Its stage-k interface label is (anc_k(dl), anc_k(dh)).  Because
// that label for every k is a function of (dl, dh) alone, the finest clusters
// are the distinct (node, dl, dh) triples; sorting those triples (level
// descending, node ascending, then the labels of stages 2..L
// lexicographically) and listing points in natural order inside each triple
// gives the permutation, and every coarser cluster is a run of triples.
#include <algorithm>
#include <array>
#include <climits>
#include <memory>
#include <numeric>

#include "common.hpp"

namespace spaqr {

namespace {

struct Tree {
  int dim, L;
  std::vector<int32_t> axis;   // split axis per internal node
  std::vector<int64_t> msplit; // split coordinate m per internal node
};

int64_t descend(const Tree& t, const int64_t* c, int64_t node) {
  while (bit_length((uint64_t)node) < t.L) {
    int ax = t.axis[node];
    int64_t m = t.msplit[node];
    int64_t v = c[ax];
    if (v == m || v == m + 1) return node;
    node = 2 * node + (v >= m + 2 ? 1 : 0);
  }
  return node;
}

struct Finest {
  int32_t level;
  int64_t node, dl, dh;
};

void finish_ordering(Ordering* o, const std::vector<Finest>& fin);

}  // namespace

Ordering* build_grid_ordering(int dim, const int32_t sides[3], int nlevels) {
  SPAQR_REQUIRE(dim == 2 || dim == 3, SPAQR_EINVAL, "dim must be 2 or 3");
  int64_t n = 1;
  for (int a = 0; a < dim; ++a) {
    SPAQR_REQUIRE(sides[a] >= 1, SPAQR_EINVAL, "grid sides must be >= 1");
    n *= sides[a];
  }
  int L = nlevels;
  if (L <= 0) {
    // smallest L with 64 * 2^L >= n, i.e. ceil(log2(n / 64)); at least 1
    L = 0;
    while ((int64_t(64) << L) < n) ++L;
    L = std::max(1, L);
    // capped at the deepest tree whose boxes above the leaves all split
    // (longest extent >= 4); the extents of a box's children follow the
    // split rule below, so the boxes of each level are simulated in turn
    std::vector<std::array<int64_t, 3>> box{{sides[0], dim > 1 ? sides[1] : 1, dim > 2 ? sides[2] : 1}};
    int depth = 1;
    while (depth < L) {
      std::vector<std::array<int64_t, 3>> next;
      bool ok = true;
      for (const auto& e : box) {
        int ax = 0;
        for (int a = 1; a < dim; ++a)
          if (e[a] > e[ax]) ax = a;
        if (e[ax] < 4) {
          ok = false;
          break;
        }
        const int64_t lw = (e[ax] - 2) / 2;
        auto c0 = e, c1 = e;
        c0[ax] = lw;
        c1[ax] = e[ax] - 2 - lw;
        next.push_back(c0);
        next.push_back(c1);
      }
      if (!ok) break;
      box.swap(next);
      ++depth;
    }
    L = std::min(L, depth);
  }
  SPAQR_REQUIRE(L >= 1 && L <= 30, SPAQR_EINVAL, "levels out of range");

  auto* o = new Ordering();
  std::unique_ptr<Ordering> guard(o);
  o->dim = dim;
  for (int a = 0; a < 3; ++a) o->sides[a] = a < dim ? sides[a] : 1;
  o->L = L;
  o->n = n;

  // ---- tree of boxes
  Tree t;
  t.dim = dim;
  t.L = L;
  const int64_t nn = int64_t(1) << L;
  t.axis.assign(nn, -1);
  t.msplit.assign(nn, -1);
  std::vector<int64_t> lo(nn * 3, 0), hi(nn * 3, 0);
  for (int a = 0; a < dim; ++a) hi[1 * 3 + a] = sides[a];
  for (int64_t b = 1; b < (int64_t(1) << (L - 1)); ++b) {
    int ax = 0;
    int64_t w = hi[b * 3] - lo[b * 3];
    for (int a = 1; a < dim; ++a) {
      int64_t e = hi[b * 3 + a] - lo[b * 3 + a];
      if (e > w) { w = e; ax = a; }
    }
    SPAQR_REQUIRE(w >= 4, SPAQR_EINVAL,
                  "too many levels: a box above the leaves has longest extent < 4");
    int64_t m = lo[b * 3 + ax] + (w - 2) / 2;
    t.axis[b] = ax;
    t.msplit[b] = m;
    for (int a = 0; a < 3; ++a) {
      lo[2 * b * 3 + a] = lo[b * 3 + a];
      hi[2 * b * 3 + a] = hi[b * 3 + a];
      lo[(2 * b + 1) * 3 + a] = lo[b * 3 + a];
      hi[(2 * b + 1) * 3 + a] = hi[b * 3 + a];
    }
    hi[2 * b * 3 + ax] = m;
    lo[(2 * b + 1) * 3 + ax] = m + 2;
  }

  // ---- per point: deepest node and (for separators) both sides' deepest nodes
  std::vector<Finest> fin(n);
  const int64_t s0 = sides[0], s1 = dim > 1 ? sides[1] : 1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3] = {i % s0, (i / s0) % s1, dim == 3 ? i / (s0 * s1) : 0};
    int64_t nd = descend(t, c, 1);
    int lv = bit_length((uint64_t)nd);
    Finest f{lv, nd, 0, 0};
    if (lv < L) {
      int ax = t.axis[nd];
      int64_t m = t.msplit[nd];
      int64_t cl[3] = {c[0], c[1], c[2]}, ch[3] = {c[0], c[1], c[2]};
      cl[ax] = m - 1;
      ch[ax] = m + 2;
      f.dl = descend(t, cl, 2 * nd);
      f.dh = descend(t, ch, 2 * nd + 1);
    }
    fin[i] = f;
  }

  finish_ordering(o, fin);
  guard.release();
  return o;
}

namespace {

// perm, the clusters of every stage and the merge parents from each point's
// (level, node, dl, dh); o->L and o->n are set
void finish_ordering(Ordering* o, const std::vector<Finest>& fin) {
  const int L = o->L;
  const int64_t n = o->n;
  // ---- distinct finest clusters: stable radix sort of the packed key
  // (node, dl, dh), L bits each, keeps points in natural order inside a run
  SPAQR_REQUIRE(L <= 21, SPAQR_EINVAL, "at most 21 levels");
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i)
    key[i] = ((uint64_t)fin[i].node << (2 * L)) | ((uint64_t)fin[i].dl << L) | (uint64_t)fin[i].dh;
  std::vector<int64_t> idx(n), tmp(n);
  std::iota(idx.begin(), idx.end(), 0);
  {
    const int bits = 3 * L + 1;
    std::vector<int64_t> cnt(1 << 16);
    for (int sh = 0; sh < bits; sh += 16) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int64_t i = 0; i < n; ++i) cnt[(key[idx[i]] >> sh) & 0xffff]++;
      int64_t sum = 0;
      for (auto& c : cnt) {
        const int64_t t = c;
        c = sum;
        sum += t;
      }
      for (int64_t i = 0; i < n; ++i) tmp[cnt[(key[idx[i]] >> sh) & 0xffff]++] = idx[i];
      idx.swap(tmp);
    }
  }
  // runs of equal keys
  std::vector<Finest> uniq;
  std::vector<int64_t> run_start;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || key[idx[i]] != key[idx[i - 1]]) {
      uniq.push_back(fin[idx[i]]);
      run_start.push_back(i);
    }
  run_start.push_back(n);
  const int64_t nf = (int64_t)uniq.size();
  auto less = [L](const Finest& a, const Finest& b) {
    if (a.level != b.level) return a.level > b.level;
    if (a.node != b.node) return a.node < b.node;
    for (int k = 2; k <= L; ++k) {
      int64_t x = anc_at(a.dl, k), y = anc_at(b.dl, k);
      if (x != y) return x < y;
      x = anc_at(a.dh, k);
      y = anc_at(b.dh, k);
      if (x != y) return x < y;
    }
    return false;
  };
  std::vector<int64_t> order(nf);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return less(uniq[x], uniq[y]); });
  std::vector<int64_t> cnt(nf + 1, 0);
  o->perm.resize(n);
  {
    int64_t p = 0;
    std::vector<Finest> sorted(nf);
    for (int64_t c = 0; c < nf; ++c) {
      const int64_t u = order[c];
      sorted[c] = uniq[u];
      for (int64_t i = run_start[u]; i < run_start[u + 1]; ++i) o->perm[p++] = idx[i];
      cnt[c + 1] = p;
    }
    uniq.swap(sorted);
  }
  o->iperm.assign(n, 0);
  for (int64_t p = 0; p < n; ++p) o->iperm[o->perm[p]] = p;

  // ---- clusters of every stage: runs of finest clusters with equal labels
  o->stages.assign(L + 1, StageClusters());
  for (int k = L; k >= 1; --k) {
    StageClusters& sc = o->stages[k];
    int64_t prevNode = -1, prevA = -1, prevB = -1;
    for (int64_t c = 0; c < nf; ++c) {
      const Finest& f = uniq[c];
      if (f.level > k) continue;
      int64_t a = f.level < k ? anc_at(f.dl, k) : 0;
      int64_t b = f.level < k ? anc_at(f.dh, k) : 0;
      if (sc.start.empty() || f.node != prevNode || a != prevA || b != prevB) {
        sc.start.push_back(cnt[c]);
        sc.end.push_back(cnt[c + 1]);
        sc.node.push_back(f.node);
        sc.level.push_back(f.level);
      } else {
        sc.end.back() = cnt[c + 1];
      }
      prevNode = f.node;
      prevA = a;
      prevB = b;
    }
  }
  for (int k = L; k >= 2; --k) {
    StageClusters& sc = o->stages[k];
    const StageClusters& up = o->stages[k - 1];
    sc.parent.assign(sc.count(), -1);
    for (int64_t c = 0; c < sc.count(); ++c) {
      if (sc.level[c] >= k) continue;
      auto it = std::upper_bound(up.start.begin(), up.start.end(), sc.start[c]);
      sc.parent[c] = (int64_t)(it - up.start.begin()) - 1;
    }
  }
  o->stages[1].parent.assign(o->stages[1].count(), -1);
}

}  // namespace


// ---------------------------------------------------------------------------
// Algebraic modified nested dissection of a square sparse matrix (Section 2.3,
// Fig. mnd), for inputs without a grid.  The paper partitions such matrices
// with a hypergraph partitioner on A; here the graph of A^T A (whose ND the
// column ordering is) is bisected between two far vertices:
//
//   * graph: i ~ j (i != j) iff some row holds entries in columns i and j;
//   * node X (vertex set V_X): in the subgraph induced on V_X, the root r
//     starts at min(V_X) and moves, up to four times, to the smallest vertex
//     of its last BFS level while that BFS has more levels; u is then the
//     smallest vertex of r's last level.  A vertex v of r's component gets
//     key d_r(v) - d_u(v) (BFS distances); the other components join the
//     high child;
//   * keys run over [kmin, kmax]; with kmax - kmin >= 3 the separator is the
//     key pair {t, t+1}, t in [kmin+1, kmax-2] minimizing (|#low - #high|,
//     |pair|, t), low (key < t) going to 2X and high (key > t+1) to 2X+1.
//     An edge changes each distance by at most one, so the pair cuts A^T A
//     inside V_X.  The pair is then thinned: its vertices with no neighbour in
//     the high part join the low part, then those with no neighbour in the
//     low part join the high part;
//   * a separator vertex q of node B touches, on each side C of B, the nodes
//     of its neighbours inside C's subtree; desc_C(q) is their deepest common
//     ancestor (C when there are none), and the stage-k interface of q is
//     (anc_k(desc_2B), anc_k(desc_2B+1)), as for grids;
//   * nlevels <= 0: ceil(log2(n/64)) (at least 1), capped at the deepest tree
//     whose nodes above the leaves all split.
namespace {

struct Graph {
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;  // sorted neighbour lists
};

Graph ata_graph(int64_t n, const int64_t* rowptr, const int32_t* col) {
  // columns' rows (the transpose's pattern)
  std::vector<int64_t> cptr(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t) cptr[col[t] + 1]++;
  for (int64_t c = 0; c < n; ++c) cptr[c + 1] += cptr[c];
  std::vector<int32_t> crow(cptr[n]);
  {
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t) crow[fill[col[t]]++] = (int32_t)r;
  }
  Graph g;
  g.ptr.assign(n + 1, 0);
  std::vector<int64_t> mark(n, -1);
  std::vector<int32_t> nb;
  for (int64_t i = 0; i < n; ++i) {
    nb.clear();
    for (int64_t u = cptr[i]; u < cptr[i + 1]; ++u) {
      const int32_t r = crow[u];
      for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t) {
        const int32_t j = col[t];
        if (j != i && mark[j] != i) {
          mark[j] = i;
          nb.push_back(j);
        }
      }
    }
    std::sort(nb.begin(), nb.end());
    g.adj.insert(g.adj.end(), nb.begin(), nb.end());
    g.ptr[i + 1] = (int64_t)g.adj.size();
  }
  return g;
}

// BFS level sets (each sorted) from root over the vertices v with
// cur[v] == X not yet marked with stamp; marks what it visits
void bfs_levels(const Graph& g, const std::vector<int64_t>& cur, int64_t X, int32_t root, std::vector<int64_t>& seen,
                int64_t stamp, std::vector<std::vector<int32_t>>& levels) {
  std::vector<int32_t> front{root};
  seen[root] = stamp;
  while (!front.empty()) {
    std::sort(front.begin(), front.end());
    levels.push_back(front);
    std::vector<int32_t> next;
    for (int32_t v : front)
      for (int64_t t = g.ptr[v]; t < g.ptr[v + 1]; ++t) {
        const int32_t w = g.adj[t];
        if (cur[w] == X && seen[w] != stamp) {
          seen[w] = stamp;
          next.push_back(w);
        }
      }
    front.swap(next);
  }
}

int64_t lca(int64_t a, int64_t b) {
  const int la = bit_length((uint64_t)a), lb = bit_length((uint64_t)b);
  if (la > lb) a >>= (la - lb);
  if (lb > la) b >>= (lb - la);
  while (a != b) {
    a >>= 1;
    b >>= 1;
  }
  return a;
}

}  // namespace

Ordering* build_graph_ordering(int64_t n, const int64_t* rowptr, const int32_t* col, int nlevels) {
  SPAQR_REQUIRE(n >= 1 && rowptr && col, SPAQR_EINVAL, "graph ordering: empty or NULL matrix");
  for (int64_t r = 0; r < n; ++r)
    for (int64_t t = rowptr[r]; t < rowptr[r + 1]; ++t)
      SPAQR_REQUIRE(col[t] >= 0 && col[t] < n, SPAQR_EINVAL, "graph ordering: column index out of range");
  const Graph g = ata_graph(n, rowptr, col);
  int L = nlevels;
  const bool cap = L <= 0;
  if (cap) {
    L = 0;
    while ((int64_t(64) << L) < n) ++L;
    L = std::max(1, L);
  }
  SPAQR_REQUIRE(L >= 1 && L <= 21, SPAQR_EINVAL, "levels out of range");
  std::vector<int64_t> cur(n, 1);  // node of each vertex so far
  std::vector<int64_t> seen(n, -1);
  int64_t stamp = 0;
  std::vector<int32_t> dr(n, 0), du(n, 0);  // distances from the two far vertices of a node
  std::vector<int8_t> side(n, 0);          // -1 low, 0 separator, 1 high within the node being split
  // vertex sets of the nodes of the current depth, ascending
  std::vector<std::vector<int32_t>> sets(1);
  sets[0].resize(n);
  std::iota(sets[0].begin(), sets[0].end(), 0);
  int depth = 1;
  while (depth < L) {
    const int64_t first = int64_t(1) << (depth - 1);
    std::vector<std::vector<int32_t>> next(2 * sets.size());
    std::vector<std::pair<int64_t, std::vector<int32_t>>> seps;
    bool ok = true;
    for (size_t xi = 0; xi < sets.size() && ok; ++xi) {
      const int64_t X = first + (int64_t)xi;
      const std::vector<int32_t>& V = sets[xi];
      if (V.empty()) {
        ok = false;
        break;
      }
      // two far vertices of the component of min(V): r moved up to four
      // times to the smallest vertex of its last BFS level, u that vertex
      std::vector<std::vector<int32_t>> lev;
      int32_t r = V[0];
      bfs_levels(g, cur, X, r, seen, ++stamp, lev);
      for (int it = 0; it < 4; ++it) {
        const int32_t u = lev.back()[0];
        std::vector<std::vector<int32_t>> lu;
        bfs_levels(g, cur, X, u, seen, ++stamp, lu);
        if (lu.size() > lev.size()) {
          r = u;
          lev.swap(lu);
        } else {
          break;
        }
      }
      const int32_t u = lev.back()[0];
      const int64_t comp_stamp = ++stamp;
      for (size_t d = 0; d < lev.size(); ++d)
        for (int32_t v : lev[d]) {
          seen[v] = comp_stamp;
          dr[v] = (int32_t)d;
        }
      {
        std::vector<std::vector<int32_t>> lu;
        bfs_levels(g, cur, X, u, seen, ++stamp, lu);
        for (size_t d = 0; d < lu.size(); ++d)
          for (int32_t v : lu[d]) du[v] = (int32_t)d;
        // the BFS from u covers the same component; restore its marks
        for (const auto& lv : lu)
          for (int32_t v : lv) seen[v] = comp_stamp;
      }
      // keys d_r - d_u over the component; the rest of V joins the high side
      int32_t kmin = INT32_MAX, kmax = INT32_MIN;
      int64_t n_other = 0;
      for (int32_t v : V) {
        if (seen[v] != comp_stamp) {
          ++n_other;
          continue;
        }
        const int32_t key = dr[v] - du[v];
        kmin = std::min(kmin, key);
        kmax = std::max(kmax, key);
      }
      if (kmax - kmin < 3) {
        ok = false;
        break;
      }
      const int h = kmax - kmin + 1;
      std::vector<int64_t> cnt(h, 0);
      for (int32_t v : V)
        if (seen[v] == comp_stamp) cnt[dr[v] - du[v] - kmin]++;
      std::vector<int64_t> below(h + 1, 0);
      for (int q = 0; q < h; ++q) below[q + 1] = below[q] + cnt[q];
      int tq = 1;
      int64_t bi = -1, bs = 0;
      for (int q = 1; q <= h - 3; ++q) {
        const int64_t lo = below[q], sp = cnt[q] + cnt[q + 1], hi = below[h] - below[q + 2] + n_other;
        const int64_t im = lo > hi ? lo - hi : hi - lo;
        if (bi < 0 || im < bi || (im == bi && sp < bs)) {
          bi = im;
          bs = sp;
          tq = q;
        }
      }
      const int32_t t = kmin + tq;
      // sides: -1 low, 0 separator, 1 high; then the separator is thinned
      for (int32_t v : V) {
        if (seen[v] != comp_stamp) {
          side[v] = 1;
          continue;
        }
        const int32_t key = dr[v] - du[v];
        side[v] = key < t ? -1 : (key > t + 1 ? 1 : 0);
      }
      for (int pass = 0; pass < 2; ++pass) {
        const int8_t want = pass == 0 ? 1 : -1, to = pass == 0 ? -1 : 1;
        std::vector<int32_t> move;
        for (int32_t v : V) {
          if (side[v] != 0) continue;
          bool touches = false;
          for (int64_t e = g.ptr[v]; e < g.ptr[v + 1] && !touches; ++e) {
            const int32_t w = g.adj[e];
            touches = cur[w] == X && side[w] == want;
          }
          if (!touches) move.push_back(v);
        }
        for (int32_t v : move) side[v] = to;
      }
      std::vector<int32_t>& lowv = next[2 * xi];
      std::vector<int32_t>& highv = next[2 * xi + 1];
      for (int32_t v : V) {
        if (side[v] < 0) lowv.push_back(v);
        else if (side[v] > 0) highv.push_back(v);
      }
    }
    if (!ok) {
      SPAQR_REQUIRE(cap, SPAQR_EINVAL, "too many levels: a node above the leaves cannot be split");
      L = depth;
      break;
    }
    for (size_t xi = 0; xi < sets.size(); ++xi) {
      const int64_t X = first + (int64_t)xi;
      for (int32_t v : next[2 * xi]) cur[v] = 2 * X;
      for (int32_t v : next[2 * xi + 1]) cur[v] = 2 * X + 1;
    }
    sets.swap(next);
    ++depth;
  }

  auto* o = new Ordering();
  std::unique_ptr<Ordering> guard(o);
  o->dim = 0;
  o->L = L;
  o->n = n;
  std::vector<Finest> fin(n);
  for (int64_t q = 0; q < n; ++q) {
    const int64_t B = cur[q];
    const int lv = bit_length((uint64_t)B);
    Finest f{lv, B, 0, 0};
    if (lv < L) {
      for (int side = 0; side < 2; ++side) {
        const int64_t C = 2 * B + side;
        const int lc = lv + 1;
        int64_t d = -1;
        for (int64_t t = g.ptr[q]; t < g.ptr[q + 1]; ++t) {
          const int64_t w = cur[g.adj[t]];
          const int lw = bit_length((uint64_t)w);
          if (lw < lc || (w >> (lw - lc)) != C) continue;
          d = d < 0 ? w : lca(d, w);
        }
        (side == 0 ? f.dl : f.dh) = d < 0 ? C : d;
      }
    }
    fin[q] = f;
  }
  finish_ordering(o, fin);
  guard.release();
  return o;
}

}  // namespace spaqr
