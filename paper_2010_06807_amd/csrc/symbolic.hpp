// Symbolic structure of a spaQR factorization: per stage, the block pattern
// over clusters, the fronts with their row and column sets and colours, the
// fill, the interface colouring and the merge map.  Everything here depends
// only on the sparsity pattern of A and the ordering, never on values.
#pragma once

#include <utility>
#include <vector>

#include "common.hpp"
#include "mem.hpp"

namespace spaqr {

using Pair = std::pair<int32_t, int32_t>;

// Row-compressed set of blocks (i, j) over the clusters of one stage.
struct BlockSet {
  int64_t nclu = 0;
  std::vector<int64_t> rowptr;  // nclu + 1
  std::vector<int32_t> col;     // sorted per row
  int64_t size() const { return (int64_t)col.size(); }
  // index of block (i, j), or -1
  int64_t find(int32_t i, int32_t j) const;
  static BlockSet from_pairs(int64_t nclu, std::vector<Pair>& pairs);  // sorts+uniques pairs
  std::vector<Pair> pairs() const;
};

struct FrontSym {
  int32_t cluster = 0;
  int32_t colour = 0;
  std::vector<int32_t> n1;    // row clusters i != s with a block (i, s), ascending
  std::vector<int32_t> cols;  // ancestor column clusters j (excluding s), ascending
  // index in the stage's `all` set of block (rows[a], cols[b]) at a * |cols'| + b,
  // rows' = [s, n1...], cols' = [s, cols...]; -1 where the block is absent
  std::vector<int64_t> blk;
};

struct IfaceSym {
  int32_t cluster = 0;
  int32_t colour = 0;
  std::vector<int32_t> rowN;  // i != p with a block (i, p), ascending
  std::vector<int32_t> colN;  // j != p with a block (p, j), ascending
  // indices in the stage's `all` set of the blocks (i, p), (p, j) and (p, p)
  // (-1 if (p, p) is absent)
  std::vector<int64_t> rowB, colB;
  int64_t ppB = -1;
};

struct StageSym {
  int k = 0;
  int64_t nclu = 0;
  BlockSet in;     // pattern at stage start
  BlockSet post;   // after the fronts (eliminated rows/cols removed, fill added)
  BlockSet all;    // in U post: every block that lives in the stage's pool
  std::vector<FrontSym> fronts;        // ascending cluster
  std::vector<int32_t> front_order;    // indices into fronts, (colour, cluster) order
  std::vector<int32_t> front_colour_ptr;  // boundaries of colours in front_order
  bool sparsify = false;
  std::vector<IfaceSym> ifaces;        // remaining clusters, ascending (if sparsify)
  std::vector<int32_t> iface_order;    // (colour, cluster) order
  std::vector<int32_t> iface_colour_ptr;
  std::vector<int32_t> remaining;      // clusters of level < k, ascending
  // merge map of the post-front blocks, in `post` order: index of the block
  // in this stage's `all` set and of its parent block in stage k-1's `all`
  // set (-1 at stage 1)
  std::vector<int64_t> post_all, post_next;
};

struct Symbolic {
  Ordering ord;                // own copy
  int L = 0, skip = 2;
  int64_t n = 0, nnz = 0;
  std::vector<StageSym> st;    // index k = 1..L
  // stage-L block storage: block t of st[L].all (row-major, its clusters'
  // sizes) starts at pool_off_L[t] of one pool of pool_off_L.back() entries
  std::vector<int64_t> pool_off_L;
  // In one host buffer (pinned when possible, so the set-up's uploads need
  // no staging copy), back to back: col_ptr (n + 1), col_nz (nnz), nz_dst
  // (nnz).  The nonzeros of A by column: column c holds entries
  // col_nz[col_ptr[c] .. col_ptr[c + 1]) of CSR order, rows ascending, for
  // column norms summed in a fixed order; nz_dst: where every nonzero of A
  // (CSR order) lands in the stage-L pool.
  HostBuffer maps;
  int64_t* col_ptr = nullptr;
  int64_t* col_nz = nullptr;
  int64_t* nz_dst = nullptr;
  size_t maps_words() const { return (size_t)(n + 1) + 2 * (size_t)nnz; }
  std::vector<int32_t> cluster_of_pos_L;  // stage-L cluster of each permuted index
  double ms_analysis = 0.0;               // host wall time of analyze()
};

Symbolic* analyze(const spaqr_csr* A, const Ordering& ord, int skip);

// Upper bound on the device bytes a factorization of S in the given precision
// (32 or 64) holds at its peak, plus the FGMRES bases of nrhs right-hand
// sides with the given restart length.
size_t device_bytes_bound(const Symbolic& S, int precision, int64_t nrhs, int restart);

}  // namespace spaqr

struct spaqr_symbolic {
  spaqr::Symbolic s;
};
