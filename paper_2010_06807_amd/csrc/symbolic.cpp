// Symbolic analysis of Algorithm 2 over the cluster hierarchy.
//
// Front of a cluster s at level k (Section 2.4): rows [s; n1(s)] where n1(s)
// are the clusters i != s holding a block (i, s); columns {s} plus the
// clusters j of proper ND ancestors of s that hold a block in some front row.
// Columns of non-ancestor clusters are left alone: H_s acts on them as the
// identity up to O(eps) (Lemma 2, Theorem well_sep).  Fill: every block
// (i, j), i in n1(s), j in the ancestor columns.
//
// Same-level fronts update a common block (i, j) only if they share a row
// cluster i and a column cluster j; greedy colouring of that conflict graph
// (ascending cluster, lowest free colour) groups fronts that touch disjoint
// blocks.  Fronts run colour by colour, ascending inside a colour.
//
// Sparsification neighbours of an interface p: blocks (i, p) and (p, j);
// interfaces that share a block are coloured apart the same way.
#include "symbolic.hpp"

#include <algorithm>
#include <chrono>
#include <memory>

namespace spaqr {

int64_t BlockSet::find(int32_t i, int32_t j) const {
  auto b = col.begin() + rowptr[i], e = col.begin() + rowptr[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it == e || *it != j) return -1;
  return (int64_t)(it - col.begin());
}

BlockSet BlockSet::from_pairs(int64_t nclu, std::vector<Pair>& pairs) {
  // bucket by row, then sort and deduplicate each (short) row
  BlockSet s;
  s.nclu = nclu;
  std::vector<int64_t> cnt(nclu + 1, 0);
  for (const Pair& p : pairs) cnt[p.first + 1]++;
  for (int64_t i = 0; i < nclu; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> tmp(pairs.size());
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (const Pair& p : pairs) tmp[pos[p.first]++] = p.second;
  }
  s.rowptr.assign(nclu + 1, 0);
  s.col.clear();
  s.col.reserve(pairs.size());
  for (int64_t i = 0; i < nclu; ++i) {
    auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
    std::sort(b, e);
    e = std::unique(b, e);
    s.col.insert(s.col.end(), b, e);
    s.rowptr[i + 1] = (int64_t)s.col.size();
  }
  return s;
}

std::vector<Pair> BlockSet::pairs() const {
  std::vector<Pair> p;
  p.reserve(col.size());
  for (int64_t i = 0; i < nclu; ++i)
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; ++t) p.emplace_back((int32_t)i, col[t]);
  return p;
}

namespace {

// Column adjacency (transpose) of a block set.
void transpose(const BlockSet& s, std::vector<int64_t>& cptr, std::vector<int32_t>& crow) {
  cptr.assign(s.nclu + 1, 0);
  for (int32_t j : s.col) cptr[j + 1]++;
  for (int64_t j = 0; j < s.nclu; ++j) cptr[j + 1] += cptr[j];
  crow.resize(s.col.size());
  std::vector<int64_t> pos(cptr.begin(), cptr.end() - 1);
  for (int64_t i = 0; i < s.nclu; ++i)
    for (int64_t t = s.rowptr[i]; t < s.rowptr[i + 1]; ++t) crow[pos[s.col[t]]++] = (int32_t)i;
}

bool sorted_intersect(const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
  size_t x = 0, y = 0;
  while (x < a.size() && y < b.size()) {
    if (a[x] == b[y]) return true;
    if (a[x] < b[y]) ++x; else ++y;
  }
  return false;
}

// Greedy colouring in index order given each item's neighbour list.
std::vector<int32_t> greedy(const std::vector<std::vector<int32_t>>& nbr) {
  std::vector<int32_t> colour(nbr.size(), -1);
  std::vector<int32_t> mark;
  for (size_t v = 0; v < nbr.size(); ++v) {
    int32_t hi = 0;
    for (int32_t u : nbr[v]) if (colour[u] >= 0) hi = std::max(hi, colour[u] + 1);
    mark.assign(hi + 1, 0);
    for (int32_t u : nbr[v]) if (colour[u] >= 0) mark[colour[u]] = 1;
    int32_t c = 0;
    while (mark[c]) ++c;
    colour[v] = c;
  }
  return colour;
}

void order_by_colour(const std::vector<int32_t>& colour, std::vector<int32_t>& order,
                     std::vector<int32_t>& ptr) {
  int32_t nc = 0;
  for (int32_t c : colour) nc = std::max(nc, c + 1);
  ptr.assign(nc + 1, 0);
  for (int32_t c : colour) ptr[c + 1]++;
  for (int32_t c = 0; c < nc; ++c) ptr[c + 1] += ptr[c];
  order.resize(colour.size());
  std::vector<int32_t> pos(ptr.begin(), ptr.end() - 1);
  for (size_t v = 0; v < colour.size(); ++v) order[pos[colour[v]]++] = (int32_t)v;
}

}  // namespace

Symbolic* analyze(const spaqr_csr* A, const Ordering& ord, int skip) {
  const auto t_start = std::chrono::steady_clock::now();
  SPAQR_REQUIRE(A && A->rowptr && A->col && A->val, SPAQR_EINVAL, "NULL matrix");
  SPAQR_REQUIRE(A->n == ord.n, SPAQR_EINVAL, "matrix size differs from the ordering");
  SPAQR_REQUIRE(A->rowptr[0] == 0 && A->rowptr[A->n] == A->nnz, SPAQR_EINVAL, "bad rowptr");
  SPAQR_REQUIRE(skip >= 0, SPAQR_EINVAL, "skip < 0");
  const int64_t n = A->n;
  for (int64_t r = 0; r < n; ++r) {
    SPAQR_REQUIRE(A->rowptr[r + 1] >= A->rowptr[r], SPAQR_EINVAL, "rowptr decreases");
    for (int64_t t = A->rowptr[r]; t < A->rowptr[r + 1]; ++t) {
      SPAQR_REQUIRE(A->col[t] >= 0 && A->col[t] < n, SPAQR_EINVAL, "column out of range");
      SPAQR_REQUIRE(t == A->rowptr[r] || A->col[t] > A->col[t - 1], SPAQR_EINVAL,
                    "columns not sorted or duplicated");
    }
  }
  auto* S = new Symbolic();
  std::unique_ptr<Symbolic> guard(S);
  S->ord = ord;
  S->L = ord.L;
  S->skip = skip;
  S->n = n;
  S->nnz = A->nnz;
  const int L = ord.L;
  S->st.assign(L + 1, StageSym());

  // ---- stage-L block pattern from the nonzeros of A
  const StageClusters& cl = ord.stages[L];
  S->cluster_of_pos_L.assign(n, 0);
  for (int64_t c = 0; c < cl.count(); ++c)
    for (int64_t p = cl.start[c]; p < cl.end[c]; ++p) S->cluster_of_pos_L[p] = (int32_t)c;
  std::vector<Pair> pairs;
  {
    // distinct column clusters of each row cluster, rows visited in perm order
    std::vector<int64_t> stamp(cl.count(), -1);
    for (int64_t c = 0; c < cl.count(); ++c)
      for (int64_t p = cl.start[c]; p < cl.end[c]; ++p) {
        const int64_t r = ord.perm[p];
        for (int64_t t = A->rowptr[r]; t < A->rowptr[r + 1]; ++t) {
          const int32_t cj = S->cluster_of_pos_L[ord.iperm[A->col[t]]];
          if (stamp[cj] != c) {
            stamp[cj] = c;
            pairs.emplace_back((int32_t)c, cj);
          }
        }
      }
  }
  BlockSet cur = BlockSet::from_pairs(cl.count(), pairs);

  for (int k = L; k >= 1; --k) {
    StageSym& ss = S->st[k];
    const StageClusters& sc = ord.stages[k];
    ss.k = k;
    ss.nclu = sc.count();
    ss.in = cur;
    std::vector<int64_t> cptr;
    std::vector<int32_t> crow;
    transpose(ss.in, cptr, crow);

    // ---- fronts
    std::vector<char> is_front(ss.nclu, 0);
    for (int64_t c = 0; c < ss.nclu; ++c)
      if (sc.level[c] == k) {
        is_front[c] = 1;
        FrontSym f;
        f.cluster = (int32_t)c;
        ss.fronts.push_back(f);
      }
    std::vector<int64_t> stamp(ss.nclu, -1);
    for (size_t fi = 0; fi < ss.fronts.size(); ++fi) {
      FrontSym& f = ss.fronts[fi];
      const int32_t s = f.cluster;
      for (int64_t t = cptr[s]; t < cptr[s + 1]; ++t)
        if (crow[t] != s) f.n1.push_back(crow[t]);
      std::sort(f.n1.begin(), f.n1.end());
      auto scan = [&](int32_t r) {
        for (int64_t t = ss.in.rowptr[r]; t < ss.in.rowptr[r + 1]; ++t) {
          int32_t j = ss.in.col[t];
          if (j == s || stamp[j] == (int64_t)fi) continue;
          stamp[j] = (int64_t)fi;
          if (is_proper_ancestor(sc.node[j], sc.node[s])) f.cols.push_back(j);
        }
      };
      scan(s);
      for (int32_t i : f.n1) scan(i);
      std::sort(f.cols.begin(), f.cols.end());
    }
    // conflict colouring: share a row cluster and a column cluster
    {
      std::vector<std::vector<int32_t>> byrow(ss.nclu);
      for (size_t fi = 0; fi < ss.fronts.size(); ++fi)
        for (int32_t i : ss.fronts[fi].n1) byrow[i].push_back((int32_t)fi);
      std::vector<std::vector<int32_t>> nbr(ss.fronts.size());
      std::vector<int64_t> seen(ss.fronts.size(), -1);
      for (size_t fi = 0; fi < ss.fronts.size(); ++fi) {
        const FrontSym& f = ss.fronts[fi];
        if (f.cols.empty()) continue;
        for (int32_t i : f.n1)
          for (int32_t g : byrow[i]) {
            if (g == (int32_t)fi || seen[g] == (int64_t)fi) continue;
            seen[g] = (int64_t)fi;
            if (sorted_intersect(f.cols, ss.fronts[g].cols)) nbr[fi].push_back(g);
          }
      }
      std::vector<int32_t> colour = greedy(nbr);
      for (size_t fi = 0; fi < ss.fronts.size(); ++fi) ss.fronts[fi].colour = colour[fi];
      order_by_colour(colour, ss.front_order, ss.front_colour_ptr);
    }
    // ---- pattern after the fronts
    {
      std::vector<Pair> post;
      for (int64_t i = 0; i < ss.nclu; ++i) {
        if (is_front[i]) continue;
        for (int64_t t = ss.in.rowptr[i]; t < ss.in.rowptr[i + 1]; ++t)
          if (!is_front[ss.in.col[t]]) post.emplace_back((int32_t)i, ss.in.col[t]);
      }
      for (const FrontSym& f : ss.fronts)
        for (int32_t i : f.n1)
          for (int32_t j : f.cols) post.emplace_back(i, j);
      std::vector<Pair> allp = post;
      ss.post = BlockSet::from_pairs(ss.nclu, post);
      std::vector<Pair> inp = ss.in.pairs();
      allp.insert(allp.end(), inp.begin(), inp.end());
      ss.all = BlockSet::from_pairs(ss.nclu, allp);
    }
    // block indices of every front's gather (pattern only: the numeric
    // planning reads them instead of searching the block set)
    for (FrontSym& f : ss.fronts) {
      const size_t nr = 1 + f.n1.size(), ncl = 1 + f.cols.size();
      f.blk.resize(nr * ncl);
      for (size_t a = 0; a < nr; ++a) {
        const int32_t i = a == 0 ? f.cluster : f.n1[a - 1];
        for (size_t b = 0; b < ncl; ++b) f.blk[a * ncl + b] = ss.all.find(i, b == 0 ? f.cluster : f.cols[b - 1]);
      }
    }
    for (int64_t c = 0; c < ss.nclu; ++c)
      if (sc.level[c] < k) ss.remaining.push_back((int32_t)c);
    // ---- interfaces
    ss.sparsify = (k <= L - skip) && (k > 1) && !ss.remaining.empty();
    if (ss.sparsify) {
      std::vector<int64_t> pptr;
      std::vector<int32_t> prow;
      transpose(ss.post, pptr, prow);
      std::vector<int32_t> idx(ss.nclu, -1);
      for (size_t t = 0; t < ss.remaining.size(); ++t) idx[ss.remaining[t]] = (int32_t)t;
      std::vector<std::vector<int32_t>> nbr(ss.remaining.size());
      for (size_t t = 0; t < ss.remaining.size(); ++t) {
        IfaceSym f;
        const int32_t p = ss.remaining[t];
        f.cluster = p;
        for (int64_t u = pptr[p]; u < pptr[p + 1]; ++u)
          if (prow[u] != p) f.rowN.push_back(prow[u]);
        for (int64_t u = ss.post.rowptr[p]; u < ss.post.rowptr[p + 1]; ++u)
          if (ss.post.col[u] != p) f.colN.push_back(ss.post.col[u]);
        for (int32_t i : f.rowN) f.rowB.push_back(ss.all.find(i, p));
        for (int32_t j : f.colN) f.colB.push_back(ss.all.find(p, j));
        f.ppB = ss.all.find(p, p);
        std::vector<int32_t> nb;
        for (int32_t q : f.rowN) nb.push_back(idx[q]);
        for (int32_t q : f.colN) nb.push_back(idx[q]);
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        SPAQR_REQUIRE(nb.empty() || nb.front() >= 0, SPAQR_EINVAL, "block to an eliminated cluster");
        nbr[t] = nb;
        ss.ifaces.push_back(std::move(f));
      }
      std::vector<int32_t> colour = greedy(nbr);
      for (size_t t = 0; t < ss.ifaces.size(); ++t) ss.ifaces[t].colour = colour[t];
      order_by_colour(colour, ss.iface_order, ss.iface_colour_ptr);
    }
    // ---- merge to stage k-1
    if (k > 1) {
      const std::vector<int64_t>& par = sc.parent;
      std::vector<Pair> up;
      up.reserve(ss.post.size());
      for (const Pair& pr : ss.post.pairs()) {
        SPAQR_REQUIRE(par[pr.first] >= 0 && par[pr.second] >= 0, SPAQR_EINVAL,
                      "block of an eliminated cluster survived the stage");
        up.emplace_back((int32_t)par[pr.first], (int32_t)par[pr.second]);
      }
      cur = BlockSet::from_pairs(ord.stages[k - 1].count(), up);
    }
  }

  // ---- merge maps (the parent stage's block set exists only now)
  for (int k = L; k >= 1; --k) {
    StageSym& ss = S->st[k];
    const int64_t np = ss.post.size();
    ss.post_all.assign(np, -1);
    ss.post_next.assign(np, -1);
    for (int64_t i = 0; i < ss.nclu; ++i)
      for (int64_t u = ss.post.rowptr[i]; u < ss.post.rowptr[i + 1]; ++u) {
        const int32_t j = ss.post.col[u];
        ss.post_all[u] = ss.all.find((int32_t)i, j);
        if (k > 1) {
          const std::vector<int64_t>& par = ord.stages[k].parent;
          ss.post_next[u] = S->st[k - 1].all.find((int32_t)par[i], (int32_t)par[j]);
        }
      }
  }

  // ---- stage-L block storage and where each nonzero lands in it
  const StageSym& sL = S->st[L];
  S->pool_off_L.assign(sL.all.size() + 1, 0);
  for (int64_t i = 0; i < sL.nclu; ++i)
    for (int64_t t = sL.all.rowptr[i]; t < sL.all.rowptr[i + 1]; ++t)
      S->pool_off_L[t + 1] = S->pool_off_L[t] + (cl.end[i] - cl.start[i]) *
                                                    (cl.end[sL.all.col[t]] - cl.start[sL.all.col[t]]);
  S->maps = HostBuffer(S->maps_words() * sizeof(int64_t));
  S->col_ptr = reinterpret_cast<int64_t*>(S->maps.data());
  S->col_nz = S->col_ptr + (n + 1);
  S->nz_dst = S->col_nz + A->nnz;
  for (int64_t r = 0; r < n; ++r) {
    int64_t pr = ord.iperm[r];
    int32_t ci = S->cluster_of_pos_L[pr];
    for (int64_t t = A->rowptr[r]; t < A->rowptr[r + 1]; ++t) {
      int64_t pc = ord.iperm[A->col[t]];
      int32_t cj = S->cluster_of_pos_L[pc];
      const int64_t b = sL.all.find(ci, cj);
      S->nz_dst[t] = S->pool_off_L[b] + (pr - cl.start[ci]) * (cl.end[cj] - cl.start[cj]) + (pc - cl.start[cj]);
    }
  }
  // ---- the nonzeros by column
  std::fill(S->col_ptr, S->col_ptr + n + 1, int64_t(0));
  for (int64_t t = 0; t < A->nnz; ++t) S->col_ptr[A->col[t] + 1]++;
  for (int64_t j = 0; j < n; ++j) S->col_ptr[j + 1] += S->col_ptr[j];
  {
    std::vector<int64_t> pos(S->col_ptr, S->col_ptr + n);
    for (int64_t t = 0; t < A->nnz; ++t) S->col_nz[pos[A->col[t]]++] = t;
  }
  S->ms_analysis = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  guard.release();
  return S;
}


// Upper bound on the device memory of one factorization and its solve.
// Ranks never exceed the cluster sizes, so every block, front and interface
// is sized here as if nothing were compressed: the stage-k cluster sizes are
// the ordering's.  Bytes are summed per arena as the engine allocates them
// (persistent factors and apply lists, per-stage workspace, the two
// ping-pong block pools) and each arena's reservation is bounded by twice
// what it hands out plus one chunk; the FGMRES bases and the apply vectors of
// nrhs right-hand sides come on top.
size_t device_bytes_bound(const Symbolic& S, int precision, int64_t nrhs, int restart) {
  const double eb = precision == 32 ? 4.0 : 8.0;
  const double n = (double)S.n, nnz = (double)S.nnz;
  const double align = 256.0;  // every arena allocation is rounded up to 256 bytes
  double persist = 8.0 * (n + 1) + 12.0 * nnz + 16.0 * n + 8.0 * align;  // CSR, column scaling, perm
  double work_peak = 8.0 * (double)S.maps_words() + align;              // set-up maps
  double pool_max = 0.0, desc_max = 0.0;
  for (int k = S.L; k >= 1; --k) {
    const StageSym& ss = S.st[k];
    const StageClusters& cl = S.ord.stages[k];
    auto sz = [&](int32_t c) { return (double)(cl.end[c] - cl.start[c]); };
    double pool = 0.0;
    for (int64_t i = 0; i < ss.all.nclu; ++i)
      for (int64_t u = ss.all.rowptr[i]; u < ss.all.rowptr[i + 1]; ++u) pool += sz((int32_t)i) * sz(ss.all.col[u]);
    pool_max = std::max(pool_max, pool * eb + align);
    double work = 0.0;
    persist += 10.0 * align;
    for (const FrontSym& F : ss.fronts) {
      double m = sz(F.cluster), kk = 0.0;
      const double nn = sz(F.cluster);
      for (int32_t i : F.n1) m += sz(i);
      for (int32_t j : F.cols) kk += sz(j);
      // V|R_ss, R_sj, tau, compact-WY panels (width <= 32), row and column
      // slot lists and the apply descriptor
      persist += eb * (m * nn + nn * kk + nn + (nn + 32.0) * 32.0) + 4.0 * (m + kk) + 128.0;
      work += eb * m * (nn + kk + 32.0) + 64.0 * (1.0 + F.n1.size()) * (1.0 + F.cols.size());
    }
    if (ss.sparsify) {
      persist += 8.0 * align;
      for (int32_t p : ss.remaining) {
        const double P = sz(p);
        // U_pp|R_pp, tau_u, panels, Q_pp, tau_q, flag, dense operators,
        // slot list and the apply descriptor
        persist += eb * (2.0 * P * P + 2.0 * P + (P + 32.0) * 32.0) + 4.0 + (P <= 64 ? 2.0 * eb * P * P : 0.0) +
                   4.0 * P + 128.0;
        work += eb * P * (P + 16.0);
      }
      for (const IfaceSym& I : ss.ifaces) {
        double m = 0.0;
        for (int32_t i : I.rowN) m += sz(i);
        for (int32_t j : I.colN) m += sz(j);
        const double P = sz(I.cluster);
        work += (eb * std::max(P, 65.0) + 16.0) * std::max(m, 1.0) + 3.0 * align + 48.0 * (I.rowN.size() + I.colN.size());
      }
      work += 64.0 * (double)ss.remaining.size() * 64.0;  // cooperative CPQR exchange buffers
    }
    // copy, QR, scaling and CPQR descriptors (the engine's own lists and
    // their concatenation by the batch driver)
    const double desc = 64.0 * (double)ss.all.size() + 128.0 * (double)(ss.fronts.size() + ss.ifaces.size());
    work += desc;
    desc_max = std::max(desc_max, desc);
    work_peak = std::max(work_peak, work);
  }
  const double chunk = 64.0 * 1048576.0;
  auto reserved = [&](double used) { return 2.0 * used + chunk; };
  const double krylov = 8.0 * n * (double)nrhs * (2.0 * restart + 8.0);  // V, Z, b, x, apply vector
  // two pool arenas (stages alternate between them), each holding one pool
  const double total = reserved(persist) + reserved(work_peak) + 2.0 * reserved(pool_max) + reserved(desc_max) + krylov;
  return (size_t)total;
}

}  // namespace spaqr
