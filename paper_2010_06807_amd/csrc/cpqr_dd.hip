// FP32 partial column-pivoted QR of the interfaces of one colour with
// downdated column norms (Sections 2.5, 2.6; rank rule of Section 4).
//
// C = [A_np^T | A_pn] (P x m, P <= 64) is factored by Businger-Golub
// pivoting stopped by the ratio rule |R_kk| >= eps |R_11|, exactly as the
// exact-norm kernels do it, with two changes to the per-step work:
//
//   * the squared tail norm of every column is downdated after each
//     reflector, ||c[k+1:]||^2 = ||c[k:]||^2 - c_k'^2 (FP64), instead of
//     being recomputed from the P - k remaining entries;
//   * a wavefront recomputes its columns' norms exactly (FP64 sums of the
//     FP32 entries) as soon as one of them has fallen below 1e-3 of its last
//     exact value (the downdate then loses digits, as LAPACK's xGEQP3 guards
//     it), and the whole workgroup recomputes and selects again before it
//     trusts a pivot whose exact norm differs from its estimate by more than
//     1 %, or before it stops.
//
// The pivot's |R_kk| used by the rank rule is always the exact norm of the
// staged pivot column, so the rank decision itself is the exact-norm one.
// One workgroup of 512 threads per interface: thread t owns columns
// t + 512 j, their rows in registers (plus, for the widest interfaces, one
// column in LDS), for the whole factorization.  One barrier per step: each
// wavefront stages its best column in LDS, and after the barrier every
// wavefront forms the same Householder vector (dlarfg convention) from the
// workgroup's winner on its own, so no second barrier is needed before the
// update.  Every row class (P rounded up to 8) is a separate unrolled body of
// the one kernel, so the interfaces of a colour take a single launch.
//
// A launch may also span several colours (DDFlow): the sequential order of
// the sparsification only orders interfaces that share a block, so an
// interface waits for its adjacent interfaces of earlier colours alone, not
// for whole colours.  Workgroups take items in ticket order from a counter,
// and every item waits only on items of smaller tickets, whose workgroups
// are already running and wait only on smaller tickets still: the waits
// cannot form a cycle, whatever the residency of the launch.  An item
// publishes its write-back and rank with an agent-scope release before it
// marks itself done; a waiter acquires before it reads them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace spaqr {

namespace {

constexpr int DD_NT = 512;          // threads per workgroup
constexpr int DD_NW = DD_NT / 64;   // wavefronts per workgroup
constexpr double DD_STALE = 1e-3;   // exact recompute below this fraction of the last exact norm^2
constexpr double DD_TRUST = 1e-2;   // largest relative gap between a pivot's estimate and its exact norm^2

// Columns per thread held in registers for a row class (rows rounded up to
// 8): the column rows plus five registers of bookkeeping each stay within
// the 256 registers of a wavefront of a 512-thread workgroup.
__host__ __device__ constexpr int dd_nc(int ps) {
  return ps <= 8 ? 12 : ps <= 16 ? 9 : ps <= 24 ? 7 : ps <= 32 ? 5 : ps <= 48 ? 4 : 3;
}
// Row classes that may keep one more column per thread in LDS.
__host__ __device__ constexpr bool dd_has_lc(int ps) { return ps == 32 || ps == 40 || ps == 56; }

template <int... Is, typename F>
__device__ __forceinline__ void dd_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<I>) for I = 0 .. N-1 (register arrays stay in registers)
template <int N, typename F>
__device__ __forceinline__ void dd_for(F&& f) {
  dd_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// Butterfly partner for offsets below 16 by DPP lane moves inside a row of
// 16 lanes (row_mirror, row_half_mirror, two quad permutations); the
// combination of the four pairings covers all 16 lanes of a row, which is
// all an all-reduce needs.  Offsets 16 and 32 are the exact xor partners,
// taken with the gfx950 lane swaps (v_permlane16_swap swaps the odd 16-lane
// rows of its first operand with the even rows of its second,
// v_permlane32_swap the upper half of the first with the lower half of the
// second), vector-ALU moves instead of an LDS round trip.
template <int OFF>
__device__ __forceinline__ int dd_partner(int v) {
  if constexpr (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((threadIdx.x & 32) ? r[0] : r[1]);
  } else if constexpr (OFF == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((threadIdx.x & 16) ? r[0] : r[1]);
  } else {
    constexpr int CTRL = OFF == 8 ? 0x140 : (OFF == 4 ? 0x141 : (OFF == 2 ? 0x4E : 0xB1));
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
  }
}
template <int OFF>
__device__ __forceinline__ double dd_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dd_partner<OFF>((int)(b & 0xffffffffLL));
  const int hi = dd_partner<OFF>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// larger norm wins, ties to the lower current position (selects, no branch)
__device__ __forceinline__ void dd_better(double ob, int op, double& b, int& p) {
  const bool w = (ob > b) | ((ob == b) & (op < p));
  b = w ? ob : b;
  p = w ? op : p;
}

template <int OFF>
__device__ __forceinline__ void dd_level(double& b, int& p) {
  dd_better(dd_partner<OFF>(b), dd_partner<OFF>(p), b, p);
}

// Sum over the wavefront, the same value on every lane (each level adds a
// pair of lanes' values in both lanes; addition commutes).
__device__ __forceinline__ double dd_wave_sum(double v) {
  v += dd_partner<32>(v);
  v += dd_partner<16>(v);
  v += dd_partner<8>(v);
  v += dd_partner<4>(v);
  v += dd_partner<2>(v);
  v += dd_partner<1>(v);
  return v;
}

// Lane k's value (k uniform), read into scalar registers.
__device__ __forceinline__ double dd_lane(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// Makes this wavefront's LDS writes visible to its own later LDS reads.
__device__ __forceinline__ void dd_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value every lane of the wavefront holds, made visibly uniform to the
// compiler (kept in scalar registers, branches on it stay scalar).
__device__ __forceinline__ int dd_uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double dd_uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// A wavefront's best column: squared norm estimate and current position.
struct DDCand {
  double nrm;
  int pos, pad;
};

// Shared-memory layout (bytes): slots 2 x NW x 64 floats, per-wavefront
// reflector NW x 64 floats, betas 64 floats, candidates 2 x NW records of 16
// bytes, neighbour offsets max_nb + 1 ints, then (16-byte aligned) the LDS
// columns: 512 threads x ps rows.
__host__ __device__ constexpr size_t dd_fixed_bytes(int max_nb) {
  return (size_t)(2 * DD_NW * 64 + DD_NW * 64 + 64) * 4 + 2 * DD_NW * sizeof(DDCand) + (size_t)(max_nb + 1) * 4;
}
__host__ __device__ constexpr size_t dd_lc_offset(int max_nb) { return (dd_fixed_bytes(max_nb) + 15) & ~size_t(15); }

struct DDShared {
  float* slot;   // 2 x NW x 64: each wavefront's best column, double-buffered
  float* vbw;    // NW x 64: each wavefront's copy of the current reflector
  float* betas;  // 64: R_kk of step k (sign included)
  DDCand* cand;  // 2 x NW: each wavefront's candidate, double-buffered
  int* off;      // max_nb + 1: first column of each neighbour block
  float4* lcol;  // rows/4 x 512: the LDS column of every thread
};

template <int PS, int NC, int LC>
__device__ __forceinline__ void cpqr_dd_body(const SpDesc<float>& d, const SpNbr* __restrict__ nb, int nnb, int m,
                                             const DDShared& sh) {
  constexpr int NCT = NC + LC;
  constexpr int NQ = PS / 4;
  const int P = dd_uni(d.P), tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double eps = dd_uni(d.eps);
  float* pool = d.pool;
  const int* off = sh.off;
  // column c of C: row ai of block (i, p) for a row neighbour, column ai of
  // block (p, j) for a column neighbour
  auto col_src = [&](int c, int64_t& str) __attribute__((always_inline)) -> float* {
    int b = 0;
    while (off[b + 1] <= c) ++b;
    const int ai = c - off[b];
    float* blk = pool + nb[b].blk;
    const int64_t ld = nb[b].ld;
    str = b < d.nrow ? 1 : ld;
    return b < d.nrow ? blk + (int64_t)ai * ld : blk + ai;
  };
  float a[NC > 0 ? NC : 1][PS];
  double nr[NCT];   // squared tail norm estimate; -1: no column, -2: pivot of an earlier step
  float nr0[NCT];   // its value at the last exact computation
  int pos[NCT];     // current position (the step index for a pivot)
  float4* lc = sh.lcol + tid;  // element q at lc[(q / 4) * DD_NT] component q % 4
  dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
    constexpr int j = decltype(J)::value;
    const int c = tid + DD_NT * j;
    pos[j] = c;
    int64_t str = 0;
    const float* src = c < m ? col_src(c, str) : nullptr;
    double s2 = 0.0;
    dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
      constexpr int q0 = 4 * decltype(Q)::value;
      float x4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x4[e] = (src && q0 + e < P) ? src[(q0 + e) * str] : 0.0f;
        s2 += (double)x4[e] * (double)x4[e];
      }
      if constexpr (j < NC) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[j][q0 + e] = x4[e];
      } else {
        lc[(q0 / 4) * DD_NT] = make_float4(x4[0], x4[1], x4[2], x4[3]);
      }
    });
    nr[j] = c < m ? s2 : -1.0;
    nr0[j] = (float)s2;
  });
  // slots j >= nsl hold no column of this interface on any thread
  const int nsl = dd_uni((m + DD_NT - 1) / DD_NT);
  // exact squared norms of rows k0.. of the live columns
  auto recompute = [&](int k0) __attribute__((always_inline)) {
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      if (j >= nsl) return;  // no column of the interface in this slot (uniform)
      double s2 = 0.0;
      dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
        constexpr int q0 = 4 * decltype(Q)::value;
        if (q0 >= P) return;  // rows beyond the interface (uniform)
        if (q0 + 3 < k0) return;
        float x4[4];
        if constexpr (j < NC) {
#pragma unroll
          for (int e = 0; e < 4; ++e) x4[e] = a[j][q0 + e];
        } else {
          const float4 l = lc[(q0 / 4) * DD_NT];
          x4[0] = l.x, x4[1] = l.y, x4[2] = l.z, x4[3] = l.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double x = (double)x4[e];
          s2 += q0 + e >= k0 ? x * x : 0.0;
        }
      });
      if (nr[j] >= 0.0) {
        nr[j] = s2;
        nr0[j] = (float)s2;
      }
    });
  };
  const int kmax = dd_uni(min(P, m));
  int k = 0, it = 0;
  double R11 = 0.0;
  bool fresh = true;  // every estimate is an exact norm (workgroup-uniform)
  bool rc = false;    // this wavefront recomputes its norms before the next selection
  while (k < kmax) {
    k = dd_uni(k);
    if (rc) recompute(k);
    rc = false;
    const int buf = it & 1;
    ++it;
    // the thread's, then the wavefront's best column; columns that are gone
    // carry negative estimates and never win
    double best = -0.5;
    int bp = INT_MAX;
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      if (j >= nsl) return;  // no column of the interface in this slot (uniform)
      dd_better(nr[j], pos[j], best, bp);
    });
    double wb = best;
    int wp = bp;
    dd_level<32>(wb, wp);
    dd_level<16>(wb, wp);
    dd_level<8>(wb, wp);
    dd_level<4>(wb, wp);
    dd_level<2>(wb, wp);
    dd_level<1>(wb, wp);
    if (wp != INT_MAX && bp == wp) {
      // the lane holding the wavefront's best column stages it
      float4* sl = reinterpret_cast<float4*>(sh.slot + (buf * DD_NW + wv) * 64);
      dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
        if (j >= nsl) return;  // no column of the interface in this slot (uniform)
        if (pos[j] == wp) {
          dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
            constexpr int qq = decltype(Q)::value;
            if constexpr (j < NC)
              sl[qq] = make_float4(a[j][4 * qq], a[j][4 * qq + 1], a[j][4 * qq + 2], a[j][4 * qq + 3]);
            else
              sl[qq] = lc[qq * DD_NT];
          });
        }
      });
    }
    if (lane == 0) sh.cand[buf * DD_NW + wv] = DDCand{wb, wp, 0};
    __syncthreads();
    int ws = 0;
    double gb = -0.5;
    int gp = INT_MAX;
#pragma unroll
    for (int w = 0; w < DD_NW; ++w) {
      const DDCand c = sh.cand[buf * DD_NW + w];
      const bool better = (c.nrm > gb) | ((c.nrm == gb) & (c.pos < gp));
      gb = better ? c.nrm : gb;
      gp = better ? c.pos : gp;
      ws = better ? w : ws;
    }
    gb = dd_uni(gb);
    gp = dd_uni(gp);
    ws = dd_uni(ws);
    if (dd_uni((int)(gp == INT_MAX))) break;  // no live column (cannot happen while k < min(P, m))
    // the winner's exact tail norm, on every wavefront
    const float* xs = sh.slot + (buf * DD_NW + ws) * 64;
    const double x = lane < P ? (double)xs[lane] : 0.0;
    const double s = dd_uni(dd_wave_sum(lane > k ? x * x : 0.0));
    const double alpha = dd_lane(x, k);
    const double n2 = alpha * alpha + s;
    const double rkk = sqrt(n2);
    if (dd_uni((int)(!fresh && (fabs(n2 - gb) > DD_TRUST * gb || (eps > 0.0 && rkk < eps * R11))))) {
      // an estimate misled the choice, or the rule would stop: select again
      // from exact norms (uniform: every wavefront saw the same values)
      rc = true;
      fresh = true;
      continue;
    }
    if (k == 0) {
      R11 = rkk;
      if (dd_uni((int)(R11 == 0.0))) break;
    }
    if (dd_uni((int)(eps > 0.0 && rkk < eps * R11))) break;
    const double beta = s == 0.0 ? alpha : -copysign(rkk, alpha);
    const double tau = s == 0.0 ? 0.0 : (beta - alpha) / beta;
    const double scal = s == 0.0 ? 1.0 : 1.0 / (alpha - beta);
    const double v = lane < k ? 0.0 : (lane == k ? 1.0 : x * scal);
    float* vb = sh.vbw + wv * 64;
    vb[lane] = (float)v;
    if (wv == 0) {
      if (lane < P) d.vq[(int64_t)lane + (int64_t)k * P] = (float)v;
      if (lane == 0) {
        d.tauq[k] = (float)tau;
        sh.betas[k] = (float)beta;
      }
    }
    // the pivot leaves the candidates (its R entries above the diagonal are
    // final; beta and the zeros below go in at the write-back); the column
    // at position k takes the pivot's old position
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      if (j >= nsl) return;  // no column of the interface in this slot (uniform)
      if (nr[j] >= 0.0) {
        if (pos[j] == gp) {
          nr[j] = -2.0;
          pos[j] = k;
        } else if (pos[j] == k) {
          pos[j] = gp;
        }
      }
    });
    dd_wave_sync();
    const float tauf = (float)tau;
    const float4* v4p = reinterpret_cast<const float4*>(vb);
    float w[NCT];
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) { w[decltype(J)::value] = 0.0f; });
    dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
      constexpr int qq = decltype(Q)::value;
      if (4 * qq >= P) return;  // rows beyond the interface (uniform)
      if (4 * qq + 3 < k) return;  // v is zero there (uniform)
      const float4 v4 = v4p[qq];
      dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
        if (j >= nsl) return;  // no column of the interface in this slot (uniform)
        if constexpr (j < NC) {
          w[j] += v4.x * a[j][4 * qq] + v4.y * a[j][4 * qq + 1] + v4.z * a[j][4 * qq + 2] + v4.w * a[j][4 * qq + 3];
        } else {
          const float4 l = lc[qq * DD_NT];
          w[j] += v4.x * l.x + v4.y * l.y + v4.z * l.z + v4.w * l.w;
        }
      });
    });
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      if (j >= nsl) return;  // no column of the interface in this slot (uniform)
      w[j] = nr[j] >= 0.0 ? tauf * w[j] : 0.0f;
    });
    dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
      constexpr int qq = decltype(Q)::value;
      if (4 * qq >= P) return;  // rows beyond the interface (uniform)
      if (4 * qq + 3 < k) return;
      const float4 v4 = v4p[qq];
      dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
        if (j >= nsl) return;  // no column of the interface in this slot (uniform)
        if constexpr (j < NC) {
          a[j][4 * qq] -= w[j] * v4.x;
          a[j][4 * qq + 1] -= w[j] * v4.y;
          a[j][4 * qq + 2] -= w[j] * v4.z;
          a[j][4 * qq + 3] -= w[j] * v4.w;
        } else {
          float4 l = lc[qq * DD_NT];
          l.x -= w[j] * v4.x;
          l.y -= w[j] * v4.y;
          l.z -= w[j] * v4.z;
          l.w -= w[j] * v4.w;
          lc[qq * DD_NT] = l;
        }
      });
    });
    // row k of every column after the update (one uniform branch)
    float ak[NCT];
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) { ak[decltype(J)::value] = 0.0f; });
    const int e = k & 3;
    dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
      constexpr int qq = decltype(Q)::value;
      if ((k >> 2) != qq) return;
      dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
        if (j >= nsl) return;  // no column of the interface in this slot (uniform)
        float y0, y1, y2, y3;
        if constexpr (j < NC) {
          y0 = a[j][4 * qq], y1 = a[j][4 * qq + 1], y2 = a[j][4 * qq + 2], y3 = a[j][4 * qq + 3];
        } else {
          const float4 l = lc[qq * DD_NT];
          y0 = l.x, y1 = l.y, y2 = l.z, y3 = l.w;
        }
        ak[j] = e == 0 ? y0 : (e == 1 ? y1 : (e == 2 ? y2 : y3));
      });
    });
    bool stale = false;
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      if (j >= nsl) return;  // no column of the interface in this slot (uniform)
      if (nr[j] >= 0.0) {
        const double y = (double)ak[j];
        nr[j] = fmax(nr[j] - y * y, 0.0);
        stale = stale || nr[j] < DD_STALE * (double)nr0[j];
      }
    });
    ++k;
    fresh = false;
    rc = __any(stale) != 0;  // this wavefront's columns only
  }
  const int r = k;
  __syncthreads();  // betas of every step visible
  if (r < P) {
    dd_for<NCT>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      const int c = tid + DD_NT * j;
      if (c >= m) return;
      int64_t str = 0;
      float* dst = col_src(c, str);
      const bool piv = nr[j] == -2.0;
      const int kp = pos[j];
      const float bk = piv ? sh.betas[kp] : 0.0f;
      dd_for<NQ>([&](auto Q) __attribute__((always_inline)) {
        constexpr int q0 = 4 * decltype(Q)::value;
        float x4[4];
        if constexpr (j < NC) {
#pragma unroll
          for (int e = 0; e < 4; ++e) x4[e] = a[j][q0 + e];
        } else {
          const float4 l = lc[(q0 / 4) * DD_NT];
          x4[0] = l.x, x4[1] = l.y, x4[2] = l.z, x4[3] = l.w;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int q = q0 + e;
          if (q < r) dst[q * str] = piv ? (q > kp ? 0.0f : (q == kp ? bk : x4[e])) : x4[e];
        }
      });
    });
    if (tid == 0) d.rank[d.cluster] = r;
  }
}

// Bound on the polls of one dependency wait (each a load and a short sleep,
// seconds in all): a wait that runs out sets *err for the host and goes on,
// so the kernel always ends.
constexpr int DD_SPIN = 1 << 24;

__device__ void cpqr_dd_item(const SpDesc<float>& d, const SpNbr* __restrict__ nbrs, int max_nb, int lc_rows,
                             bool flow);

__global__ void __launch_bounds__(DD_NT) k_cpqr_dd(const SpDesc<float>* __restrict__ descs,
                                                   const SpNbr* __restrict__ nbrs, int max_nb, int lc_rows,
                                                   DDFlow fl) {
  __shared__ int s_item;
  int item = blockIdx.x;
  if (fl.ticket) {
    if (threadIdx.x == 0) {
      const int t = __hip_atomic_fetch_add(fl.ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int q0 = fl.pred_ptr[t], q1 = fl.pred_ptr[t + 1];
      for (int q = q0; q < q1; ++q) {
        const int* f = fl.done + fl.pred[q];
        for (int spin = 0; __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0; ++spin) {
          if (spin >= DD_SPIN) {
            __hip_atomic_store(fl.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      // an item that waited on nothing reads only what the launch found
      if (q1 > q0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      s_item = t;
    }
    __syncthreads();
    item = dd_uni(s_item);
  }
  const SpDesc<float> d = descs[item];
  cpqr_dd_item(d, nbrs, max_nb, lc_rows, fl.ticket != nullptr);
  // every thread's stores, then the done mark, for an item that a later
  // item waits on (fl.succ[item] != 0)
  if (fl.ticket && dd_uni(fl.succ[item]) != 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(fl.done + item, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ void cpqr_dd_item(const SpDesc<float>& d, const SpNbr* __restrict__ nbrs, int max_nb, int lc_rows,
                             bool flow) {
  if (d.P == 0 || *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  DDShared sh;
  sh.slot = reinterpret_cast<float*>(smem);
  sh.vbw = sh.slot + 2 * DD_NW * 64;
  sh.betas = sh.vbw + DD_NW * 64;
  sh.cand = reinterpret_cast<DDCand*>(sh.betas + 64);
  sh.off = reinterpret_cast<int*>(sh.cand + 2 * DD_NW);
  sh.lcol = reinterpret_cast<float4*>(smem + dd_lc_offset(max_nb));
  const int nnb = d.nrow + d.ncol;
  const SpNbr* nb = nbrs + d.nb;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int b = 0; b < nnb; ++b) {
      sh.off[b] = o;
      // ranks of earlier items of a dataflow launch change during it
      o += flow ? __hip_atomic_load(d.rank + nb[b].cluster, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                : d.rank[nb[b].cluster];
    }
    sh.off[nnb] = o;
  }
  __syncthreads();
  const int m = dd_uni(sh.off[nnb]);
  const int ps = (d.P + 7) & ~7;
  // the host sized the launch so that m fits the class's registers, or its
  // registers plus one LDS column when lc_rows >= ps
  const bool use_lc = m > DD_NT * dd_nc(ps) && dd_has_lc(ps) && lc_rows >= ps;
  switch (ps) {
    case 8: cpqr_dd_body<8, dd_nc(8), 0>(d, nb, nnb, m, sh); break;
    case 16: cpqr_dd_body<16, dd_nc(16), 0>(d, nb, nnb, m, sh); break;
    case 24: cpqr_dd_body<24, dd_nc(24), 0>(d, nb, nnb, m, sh); break;
    case 32:
      if (use_lc) cpqr_dd_body<32, dd_nc(32), 1>(d, nb, nnb, m, sh);
      else cpqr_dd_body<32, dd_nc(32), 0>(d, nb, nnb, m, sh);
      break;
    case 40:
      if (use_lc) cpqr_dd_body<40, dd_nc(40), 1>(d, nb, nnb, m, sh);
      else cpqr_dd_body<40, dd_nc(40), 0>(d, nb, nnb, m, sh);
      break;
    case 48: cpqr_dd_body<48, dd_nc(48), 0>(d, nb, nnb, m, sh); break;
    case 56:
      if (use_lc) cpqr_dd_body<56, dd_nc(56), 1>(d, nb, nnb, m, sh);
      else cpqr_dd_body<56, dd_nc(56), 0>(d, nb, nnb, m, sh);
      break;
    case 64: cpqr_dd_body<64, dd_nc(64), 0>(d, nb, nnb, m, sh); break;
    default: break;
  }
}

}  // namespace

// Largest neighbour-column count an interface of P unknowns may have for
// this kernel (0: P outside its range).
int sparsify_dd_capacity(int P) {
  if (P < 1 || P > 64) return 0;
  const int ps = (P + 7) & ~7;
  return DD_NT * (dd_nc(ps) + (dd_has_lc(ps) ? 1 : 0));
}

// LDS rows per thread a launch must provide for an interface of P unknowns
// and at most mmax columns (0: registers suffice).
int sparsify_dd_lc_rows(int P, int mmax) {
  const int ps = (P + 7) & ~7;
  return mmax > DD_NT * dd_nc(ps) ? ps : 0;
}

void launch_sparsify_dd(const SpDesc<float>* d, int64_t n, const SpNbr* nb, int max_nb, int lc_rows, hipStream_t s,
                        const DDFlow* flow) {
  if (n <= 0) return;
  const DDFlow fl = flow ? *flow : DDFlow{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  const size_t lds = dd_lc_offset(max_nb) + (size_t)lc_rows * DD_NT * sizeof(float);
  if (lds > 64 * 1024) {
    static std::mutex mu;
    static size_t set = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (lds > set) {
      int dev = 0, lim = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lim <= 0)
        lim = 64 * 1024;
      if (lds > (size_t)lim) throw Error(SPAQR_ENOMEM, "k_cpqr_dd: LDS need exceeds the device limit");
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cpqr_dd), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds) != hipSuccess)
        throw Error(SPAQR_EDEVICE, "k_cpqr_dd: cannot raise the LDS limit");
      set = lds;
    }
  }
  count_launch("k_cpqr_dd");
  hipLaunchKernelGGL(k_cpqr_dd, dim3((unsigned)n), dim3(DD_NT), lds, s, d, nb, max_nb, lc_rows, fl);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string("launch of k_cpqr_dd failed: ") + hipGetErrorString(e));
}

}  // namespace spaqr
