// Shared host-side definitions of the spaQR engine.
#pragma once

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "spaqr.h"

namespace spaqr {

// Error carried to the ABI boundary, where it becomes a status code.
struct Error : std::runtime_error {
  int status;
  Error(int s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define SPAQR_REQUIRE(cond, status, msg)                 \
  do {                                                   \
    if (!(cond)) throw ::spaqr::Error((status), (msg));  \
  } while (0)

inline int bit_length(uint64_t v) { return v ? 64 - __builtin_clzll(v) : 0; }

// Level-k ancestor of heap node x (x itself if level(x) <= k).
inline int64_t anc_at(int64_t x, int k) {
  int lx = bit_length((uint64_t)x);
  return lx > k ? (x >> (lx - k)) : x;
}

// True if heap node a is a proper ancestor of heap node b.
inline bool is_proper_ancestor(int64_t a, int64_t b) {
  int la = bit_length((uint64_t)a), lb = bit_length((uint64_t)b);
  return la < lb && (b >> (lb - la)) == a;
}

// ---------------------------------------------------------------- ordering
struct StageClusters {
  std::vector<int64_t> start, end, node;
  std::vector<int32_t> level;
  std::vector<int64_t> parent;  // index in the stage-(k-1) list, -1 if eliminated
  int64_t count() const { return (int64_t)start.size(); }
};

struct Ordering {
  int dim = 0;
  int32_t sides[3] = {1, 1, 1};
  int L = 0;
  int64_t n = 0;
  std::vector<int64_t> perm;          // new -> old
  std::vector<int64_t> iperm;         // old -> new
  std::vector<StageClusters> stages;  // index k (1..L); [0] unused
};

Ordering* build_grid_ordering(int dim, const int32_t sides[3], int nlevels);
Ordering* build_graph_ordering(int64_t n, const int64_t* rowptr, const int32_t* col, int nlevels);

// Process-wide kernel dispatch thresholds (spaqr_tuning); read when a stage
// is planned and launched.
const spaqr_tuning& tuning();

}  // namespace spaqr

struct spaqr_ordering {
  spaqr::Ordering o;
};
