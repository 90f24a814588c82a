// FP32 partial column-pivoted QR of wide interfaces by a team of workgroups
// (Sections 2.5, 2.6; rank rule of Section 4).
//
// The 3D interfaces near the top of the tree have up to ~900 unknowns and
// tens of thousands of neighbour columns: C = [A_np^T | A_pn] does not fit
// one workgroup.  A team of T workgroups (one per compute unit, 512 threads
// each) keeps all of C in registers for the whole factorization:
//
//   * wavefront w of team member g owns the NCW columns
//     c = (8 g + w) NCW + j, j < NCW, and lane l of it holds rows l + 64 i,
//     i < R, of each (so P <= 64 R);
//   * the per-column scalars (squared norm estimate, its last exact value,
//     the current position) of column j live in lane j << SH of its
//     wavefront (SH = 6 - log2 JB, JB = NCW rounded up to a power of two),
//     where the reduce-scatter of the column dots leaves column j's dot
//     (dots and column norms are reduced in FP32, the norm estimates kept
//     and downdated in FP64).
//
// One pivot step: every wavefront finds its best column (wavefront argmax),
// every workgroup its best (through LDS), and every member publishes its
// best column's norm, position and values in a double-buffered global slot;
// one team barrier; every member reads the T candidates, takes the same
// winner, reads its values and forms the same Householder vector (dlarfg
// convention); every wavefront updates its columns: partial dots over its R
// rows, one reduce-scatter for all NCW columns, the scaled dots broadcast
// with readlane, the rank-one update, and the squared norms downdated in
// FP64 from the new row k.  Norms are recomputed exactly when one has lost
// three digits, and by the whole team before it stops or trusts an estimate
// that differs from the winner's exact norm by more than 1 % (the same rules
// as the single-workgroup downdated kernel), so the rank decision always
// uses the exact norm of the chosen pivot.
//
// The members of a team must be co-resident (cooperative launch); each team
// has its own barrier counters, so teams of one launch never wait for each
// other, and a team's members leave together after the write-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace spaqr {

namespace {

constexpr int TM_NT = 512;
constexpr int TM_NW = TM_NT / 64;
constexpr int TM_PMAX = 896;         // rows of the largest class (R = 14)
constexpr double TM_STALE = 1e-3;    // exact recompute below this fraction of the last exact norm^2
constexpr double TM_TRUST = 1e-2;    // largest relative gap between a pivot's estimate and its exact norm^2

template <int... Is, typename F>
__device__ __forceinline__ void tm_for_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
// f(integral_constant<I>) for I = 0 .. N-1 (register arrays stay in registers)
template <int N, typename F>
__device__ __forceinline__ void tm_for(F&& f) {
  tm_for_impl(std::make_integer_sequence<int, N>{}, f);
}

__host__ __device__ constexpr int tm_log2(int x) { return x <= 1 ? 0 : 1 + tm_log2(x / 2); }
__host__ __device__ constexpr int tm_pow2(int x) { return x <= 1 ? 1 : 2 * tm_pow2((x + 1) / 2); }

// Partner lane for a butterfly level: DPP lane moves inside a row of 16 lanes
// for offsets below 16 (row_mirror, row_half_mirror, two quad permutations;
// together they cover a row); the exact xor partners for 16 and 32 by the
// gfx950 lane swaps (v_permlane16_swap: odd 16-lane rows of the first
// operand with even rows of the second; v_permlane32_swap: upper half of the
// first with lower half of the second), vector-ALU moves, no LDS.
template <int OFF>
__device__ __forceinline__ int tm_partner(int v) {
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
__device__ __forceinline__ float tm_partner(float v) {
  return __int_as_float(tm_partner<OFF>(__float_as_int(v)));
}
template <int OFF>
__device__ __forceinline__ double tm_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = tm_partner<OFF>((int)(b & 0xffffffffLL));
  const int hi = tm_partner<OFF>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ int tm_uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double tm_uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ float tm_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// larger norm wins, ties to the lower current position
__device__ __forceinline__ void tm_better(double ob, int op, double& b, int& p) {
  const bool w = (ob > b) | ((ob == b) & (op < p));
  b = w ? ob : b;
  p = w ? op : p;
}
template <int OFF>
__device__ __forceinline__ void tm_level(double& b, int& p) {
  tm_better(tm_partner<OFF>(b), tm_partner<OFF>(p), b, p);
}
__device__ __forceinline__ void tm_wave_argmax(double& b, int& p) {
  tm_level<32>(b, p);
  tm_level<16>(b, p);
  tm_level<8>(b, p);
  tm_level<4>(b, p);
  tm_level<2>(b, p);
  tm_level<1>(b, p);
}

__device__ __forceinline__ double tm_wave_sum(double v) {
  v += tm_partner<32>(v);
  v += tm_partner<16>(v);
  v += tm_partner<8>(v);
  v += tm_partner<4>(v);
  v += tm_partner<2>(v);
  v += tm_partner<1>(v);
  return v;
}

// One butterfly level of the reduce-scatter of H2 = 2 H values: lanes with
// bit OFF set keep the upper half.
template <typename T, int H, int OFF, int N>
__device__ __forceinline__ void tm_rs_level(T (&v)[N], int lane) {
  if constexpr (H >= 1) {
    const bool hi = (lane & OFF) != 0;
    tm_for<H>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const T lo_v = v[i], hi_v = v[i + H];
      const T send = hi ? lo_v : hi_v;
      const T keep = hi ? hi_v : lo_v;
      v[i] = keep + tm_partner<OFF>(send);
    });
    tm_rs_level<T, H / 2, OFF / 2, N>(v, lane);
  }
}
// v[JB] per lane -> every lane holds the wavefront total of value index
// lane >> (6 - log2 JB).
template <typename T, int JB>
__device__ __forceinline__ T tm_reduce_scatter(T (&v)[JB]) {
  const int lane = threadIdx.x & 63;
  tm_rs_level<T, JB / 2, 32, JB>(v, lane);
  T s = v[0];
  constexpr int OFF0 = 32 >> tm_log2(JB);
  if constexpr (OFF0 >= 32) s += tm_partner<32>(s);
  if constexpr (OFF0 >= 16) s += tm_partner<16>(s);
  if constexpr (OFF0 >= 8) s += tm_partner<8>(s);
  if constexpr (OFF0 >= 4) s += tm_partner<4>(s);
  if constexpr (OFF0 >= 2) s += tm_partner<2>(s);
  if constexpr (OFF0 >= 1) s += tm_partner<1>(s);
  return s;
}

// Barrier of the nblk members of one team (agent-scope release/acquire; the
// workgroup barrier first orders every wavefront's stores before thread 0's
// release).
// The wait is bounded (about 2^27 short sleeps, seconds): a member that runs
// out of it leaves the barrier anyway, so the kernel always ends; *err then
// records it for the host.
__device__ __forceinline__ void tm_team_sync(int* cnt, int* gen, int nblk, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(cnt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nblk - 1) {
      __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // relaxed polling (no cache invalidation per poll), one acquire after
      for (int spin = 0; __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g; ++spin) {
        if (spin >= (1 << 27)) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// Team-wide scratch of one launch (global memory, the caller zeroes sync).
struct TeamBuf {
  double* cn;   // 2 x total: candidate squared norms
  int* cp;      // 2 x total: candidate positions
  float* cv;    // 2 x total x TM_PMAX: candidate column values
  int* sync;    // 2 per team: arrival count, generation
  int* err;     // set when a barrier wait ran out (results of that launch invalid)
  int total;    // workgroups the candidate arrays are laid out for
};

// Shared memory of a workgroup.
struct TeamShared {
  double wn[2][TM_NW];    // per-wavefront candidates, double-buffered
  int wp[2][TM_NW];
  int wj[2][TM_NW];       // the candidate's column slot within its wavefront
  double red[TM_NW];      // team-candidate reduction
  int redp[TM_NW], redg[TM_NW];
  float betas[TM_PMAX];   // R_kk of every step (sign included)
  int off[1];             // neighbour offsets (max_nb + 1), sized at launch
};

template <int R, int NCW>
__device__ __forceinline__ void cpqr_team_body(const SpDesc<float>& d, const SpNbr* __restrict__ nb, int nnb, int m,
                                               int g, int T, int base, const TeamBuf tb, int* cnt, int* gen,
                                               TeamShared& sh) {
  constexpr int JB = tm_pow2(NCW);
  constexpr int SH = 6 - tm_log2(JB);
  const int P = tm_uni(d.P), tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double eps = tm_uni(d.eps);
  float* pool = d.pool;
  const int* off = sh.off;
  auto col_src = [&](int c, int64_t& str) __attribute__((always_inline)) -> float* {
    int b = 0;
    while (off[b + 1] <= c) ++b;
    const int ai = c - off[b];
    float* blk = pool + nb[b].blk;
    const int64_t ld = nb[b].ld;
    str = b < d.nrow ? 1 : ld;
    return b < d.nrow ? blk + (int64_t)ai * ld : blk + ai;
  };
  const int c0 = (g * TM_NW + wv) * NCW;  // first column of this wavefront
  // this lane's column slot (valid for lanes whose low SH bits are zero and
  // whose slot is below NCW)
  const int myj = lane >> SH;
  const bool owner = (lane & ((1 << SH) - 1)) == 0 && myj < NCW;
  float a[NCW][R];
  double nr = -1.0;  // owner lanes: squared tail norm estimate; -1: no column, -2: pivot of an earlier step
  float nr0 = 0.0f;  // its last exact value
  int pos = INT_MAX; // current position (the step index for a pivot)
  {
    float part[JB];
    tm_for<JB>([&](auto J) __attribute__((always_inline)) { part[decltype(J)::value] = 0.0f; });
    tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      const int c = c0 + j;
      int64_t str = 0;
      const float* src = c < m ? col_src(c, str) : nullptr;
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const int q = lane + 64 * i;
        const float x = (src && q < P) ? src[q * str] : 0.0f;
        a[j][i] = x;
        part[j] += x * x;
      });
    });
    const float s2 = tm_reduce_scatter<float, JB>(part);
    if (owner && c0 + myj < m) {
      nr = (double)s2;
      nr0 = s2;
      pos = c0 + myj;
    }
  }
  // exact squared norms of rows k0.. of the live columns of this wavefront
  auto recompute = [&](int k0) __attribute__((always_inline)) {
    float part[JB];
    tm_for<JB>([&](auto J) __attribute__((always_inline)) { part[decltype(J)::value] = 0.0f; });
    tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const float x = a[j][i];
        part[j] += lane + 64 * i >= k0 ? x * x : 0.0f;
      });
    });
    const float s2 = tm_reduce_scatter<float, JB>(part);
    if (owner && nr >= 0.0) {
      nr = (double)s2;
      nr0 = s2;
    }
  };
  const int kmax = tm_uni(min(P, m));
  int k = 0, it = 0;
  double R11 = 0.0;
  bool fresh = true;  // every estimate is an exact norm (team-uniform)
  bool rc = false;    // this wavefront recomputes before the next selection
  while (k < kmax) {
    k = tm_uni(k);
    if (rc) recompute(k);
    rc = false;
    const int buf = it & 1;
    ++it;
    // wavefront and workgroup candidates
    {
      double b = owner && nr >= 0.0 ? nr : -0.5;
      int p = owner && nr >= 0.0 ? pos : INT_MAX;
      tm_wave_argmax(b, p);
      const unsigned long long hit = __ballot(owner && nr >= 0.0 && pos == p);
      if (lane == 0) {
        sh.wn[buf][wv] = b;
        sh.wp[buf][wv] = p;
        sh.wj[buf][wv] = hit ? (int)(__builtin_ctzll(hit) >> SH) : 0;
      }
    }
    __syncthreads();
    double gbw = -0.5;
    int gpw = INT_MAX, gww = 0;
#pragma unroll
    for (int w = 0; w < TM_NW; ++w) {
      const double ob = sh.wn[buf][w];
      const int op = sh.wp[buf][w];
      const bool better = (ob > gbw) | ((ob == gbw) & (op < gpw));
      gbw = better ? ob : gbw;
      gpw = better ? op : gpw;
      gww = better ? w : gww;
    }
    gww = tm_uni(gww);
    // publish this member's candidate: norm, position and the column values
    // (written by the wavefront that owns it)
    {
      const int slot = buf * tb.total + base + g;
      if (tid == 0) {
        tb.cn[slot] = gbw;
        tb.cp[slot] = gpw;
      }
      if (wv == gww && gpw != INT_MAX) {
        const int jw = tm_uni(sh.wj[buf][gww]);
        float* dst = tb.cv + (size_t)slot * TM_PMAX;
        tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
          constexpr int j = decltype(J)::value;
          if (j != jw) return;  // uniform
          tm_for<R>([&](auto I) __attribute__((always_inline)) {
            constexpr int i = decltype(I)::value;
            const int q = lane + 64 * i;
            if (q < P) dst[q] = a[j][i];
          });
        });
      }
    }
    tm_team_sync(cnt, gen, T, tb.err);
    // the team's winner, identically on every member
    {
      double b = -0.5;
      int p = INT_MAX, gw = 0;
      for (int t = tid; t < T; t += TM_NT) {
        const double ob = tb.cn[buf * tb.total + base + t];
        const int op = tb.cp[buf * tb.total + base + t];
        const bool better = (ob > b) | ((ob == b) & (op < p));
        b = better ? ob : b;
        p = better ? op : p;
        gw = better ? t : gw;
      }
      // wavefront argmax carrying the member index
      tm_for<6>([&](auto L) __attribute__((always_inline)) {
        constexpr int OFF = 32 >> decltype(L)::value;
        const double ob = tm_partner<OFF>(b);
        const int op = tm_partner<OFF>(p);
        const int og = tm_partner<OFF>(gw);
        const bool better = (ob > b) | ((ob == b) & (op < p));
        b = better ? ob : b;
        p = better ? op : p;
        gw = better ? og : gw;
      });
      if (lane == 0) {
        sh.red[wv] = b;
        sh.redp[wv] = p;
        sh.redg[wv] = gw;
      }
    }
    __syncthreads();
    double gb = -0.5;
    int gp = INT_MAX, gg = 0;
#pragma unroll
    for (int w = 0; w < TM_NW; ++w) {
      const double ob = sh.red[w];
      const int op = sh.redp[w];
      const bool better = (ob > gb) | ((ob == gb) & (op < gp));
      gb = better ? ob : gb;
      gp = better ? op : gp;
      gg = better ? sh.redg[w] : gg;
    }
    gb = tm_uni(gb);
    gp = tm_uni(gp);
    gg = tm_uni(gg);
    if (tm_uni((int)(gp == INT_MAX))) break;  // no live column (cannot happen while k < min(P, m))
    // the winner's values and its exact tail norm (every wavefront)
    float x[R];
    double s = 0.0, alpha = 0.0;
    {
      const float* src = tb.cv + (size_t)(buf * tb.total + base + gg) * TM_PMAX;
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const int q = lane + 64 * i;
        x[i] = q < P ? src[q] : 0.0f;
        s += q > k ? (double)x[i] * (double)x[i] : 0.0;
      });
      s = tm_uni(tm_wave_sum(s));
      const int sk = k >> 6, lk = k & 63;
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        if (i == sk) alpha = (double)tm_lane(x[i], lk);
      });
      alpha = tm_uni(alpha);
    }
    const double n2 = alpha * alpha + s;
    const double rkk = sqrt(n2);
    if (tm_uni((int)(!fresh && (fabs(n2 - gb) > TM_TRUST * gb || (eps > 0.0 && rkk < eps * R11))))) {
      // an estimate misled the choice, or the rule would stop: select again
      // from exact norms (uniform over the team: all saw the same values)
      rc = true;
      fresh = true;
      continue;
    }
    if (k == 0) {
      R11 = rkk;
      if (tm_uni((int)(R11 == 0.0))) break;
    }
    if (tm_uni((int)(eps > 0.0 && rkk < eps * R11))) break;
    const double beta = s == 0.0 ? alpha : -copysign(rkk, alpha);
    const double tau = s == 0.0 ? 0.0 : (beta - alpha) / beta;
    const double scal = s == 0.0 ? 1.0 : 1.0 / (alpha - beta);
    float v[R];
    tm_for<R>([&](auto I) __attribute__((always_inline)) {
      constexpr int i = decltype(I)::value;
      const int q = lane + 64 * i;
      v[i] = q < k ? 0.0f : (q == k ? 1.0f : (float)((double)x[i] * scal));
    });
    if (g == 0 && wv == 0) {
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const int q = lane + 64 * i;
        if (q < P) d.vq[(int64_t)q + (int64_t)k * P] = v[i];
      });
      if (lane == 0) d.tauq[k] = (float)tau;
    }
    if (tid == 0) sh.betas[k] = (float)beta;
    // the pivot leaves the candidates (beta and the zeros below go in at the
    // write-back); the column at position k takes the pivot's old position
    if (owner && nr >= 0.0) {
      if (pos == gp) {
        nr = -2.0;
        pos = k;
      } else if (pos == k) {
        pos = gp;
      }
    }
    // update: partial dots, one reduce-scatter, scaled dots by readlane
    float w;
    {
      float part[JB];
      tm_for<JB>([&](auto J) __attribute__((always_inline)) { part[decltype(J)::value] = 0.0f; });
      tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
        constexpr int j = decltype(J)::value;
        float acc = 0.0f;
        tm_for<R>([&](auto I) __attribute__((always_inline)) {
          constexpr int i = decltype(I)::value;
          acc += v[i] * a[j][i];
        });
        part[j] = acc;
      });
      w = tm_reduce_scatter<float, JB>(part);
    }
    const float tw = owner && nr >= 0.0 ? (float)tau * w : 0.0f;
    tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      const float t = tm_lane(tw, j << SH);
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        a[j][i] -= t * v[i];
      });
    });
    // row k of every column after the update, to its owner lane
    float ak = 0.0f;
    {
      const int sk = k >> 6, lk = k & 63;
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        if (i != sk) return;  // uniform
        tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
          constexpr int j = decltype(J)::value;
          const float y = tm_lane(a[j][i], lk);
          ak = myj == j ? y : ak;
        });
      });
    }
    bool stale = false;
    if (owner && nr >= 0.0) {
      const double y = (double)ak;
      nr = fmax(nr - y * y, 0.0);
      stale = nr < TM_STALE * (double)nr0;
    }
    ++k;
    fresh = false;
    rc = __any(stale) != 0;  // this wavefront's columns only
  }
  const int r = k;
  __syncthreads();  // betas visible
  if (r < P) {
    // pivots: beta at their step's row and zeros below; the others as updated
    tm_for<NCW>([&](auto J) __attribute__((always_inline)) {
      constexpr int j = decltype(J)::value;
      const int c = c0 + j;
      if (c >= m) return;  // uniform
      const int src_lane = j << SH;
      const double cn = __shfl(nr, src_lane, 64);
      const int kp = __shfl(pos, src_lane, 64);
      const bool piv = cn == -2.0;
      const float bk = piv ? sh.betas[kp] : 0.0f;
      int64_t str = 0;
      float* dst = col_src(c, str);
      tm_for<R>([&](auto I) __attribute__((always_inline)) {
        constexpr int i = decltype(I)::value;
        const int q = lane + 64 * i;
        if (q < r) dst[q * str] = piv ? (q > kp ? 0.0f : (q == kp ? bk : a[j][i])) : a[j][i];
      });
    });
    if (g == 0 && tid == 0) d.rank[d.cluster] = r;
  }
}

__global__ void __launch_bounds__(TM_NT) k_cpqr_team(const SpDesc<float>* __restrict__ descs,
                                                     const SpNbr* __restrict__ nbrs, const CoopItem* __restrict__ items,
                                                     int nitems, TeamBuf tb) {
  extern __shared__ __align__(16) unsigned char smem[];
  TeamShared& sh = *reinterpret_cast<TeamShared*>(smem);
  const int b = blockIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  const int itm = tm_uni(lo);
  const CoopItem ci = items[itm];
  const SpDesc<float> d = descs[itm];
  const int g = b - ci.first, T = ci.nblk, base = ci.first;
  int* cnt = tb.sync + 2 * itm;
  int* gen = cnt + 1;
  if (d.P == 0 || *d.flag != 0) return;  // the whole team returns: nobody waits
  const int nnb = d.nrow + d.ncol;
  const SpNbr* nb = nbrs + d.nb;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int q = 0; q < nnb; ++q) {
      sh.off[q] = o;
      o += d.rank[nb[q].cluster];
    }
    sh.off[nnb] = o;
  }
  __syncthreads();
  const int m = tm_uni(sh.off[nnb]);
  const int P = d.P;
  if (P <= 64) cpqr_team_body<1, 64>(d, nb, nnb, m, g, T, base, tb, cnt, gen, sh);
  else if (P <= 128) cpqr_team_body<2, 48>(d, nb, nnb, m, g, T, base, tb, cnt, gen, sh);
  else if (P <= 256) cpqr_team_body<4, 32>(d, nb, nnb, m, g, T, base, tb, cnt, gen, sh);
  else if (P <= 512) cpqr_team_body<8, 16>(d, nb, nnb, m, g, T, base, tb, cnt, gen, sh);
  else cpqr_team_body<14, 10>(d, nb, nnb, m, g, T, base, tb, cnt, gen, sh);
}

__host__ __device__ constexpr int tm_cols_per_block(int P) {
  return TM_NW * (P <= 64 ? 64 : P <= 128 ? 48 : P <= 256 ? 32 : P <= 512 ? 16 : 10);
}

}  // namespace

// Workgroups a team needs for an interface of P unknowns and at most mmax
// columns (0: P outside the kernel's range).
int sparsify_team_blocks(int P, int mmax) {
  if (P < 1 || P > TM_PMAX) return 0;
  return std::max(1, (mmax + tm_cols_per_block(P) - 1) / tm_cols_per_block(P));
}

// Workgroups one launch may hold (all co-resident), for max_nb neighbours.
int sparsify_team_capacity(int max_nb) {
  const size_t lds = sizeof(TeamShared) + (size_t)(max_nb + 1) * sizeof(int);
  int per_cu = 0, dev = 0, cus = 0;
  if (lds > 64 * 1024) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_cpqr_team), TM_NT,
                                                   lds) != hipSuccess)
    return 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

size_t sparsify_team_cand_bytes(int max_blocks) {
  return (size_t)2 * max_blocks * (sizeof(double) + sizeof(int) + (size_t)TM_PMAX * sizeof(float)) + 256;
}

bool launch_sparsify_team(const SpDesc<float>* d, const CoopItem* items, int nitems, int total_blocks,
                          const SpNbr* nb, int max_nb, int* sync, void* cand, int cand_blocks, int* err,
                          hipStream_t s) {
  if (nitems <= 0) return true;
  if (total_blocks > cand_blocks || total_blocks > sparsify_team_capacity(max_nb)) return false;
  TeamBuf tb;
  char* p = static_cast<char*>(cand);
  tb.cn = reinterpret_cast<double*>(p);
  p += (size_t)2 * cand_blocks * sizeof(double);
  tb.cv = reinterpret_cast<float*>(p);
  p += (size_t)2 * cand_blocks * TM_PMAX * sizeof(float);
  tb.cp = reinterpret_cast<int*>(p);
  tb.err = err;
  tb.sync = sync;
  tb.total = cand_blocks;
  const size_t lds = sizeof(TeamShared) + (size_t)(max_nb + 1) * sizeof(int);
  void* args[] = {(void*)&d, (void*)&nb, (void*)&items, (void*)&nitems, (void*)&tb};
  count_launch("k_cpqr_team");
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_cpqr_team), dim3((unsigned)total_blocks),
                                                  dim3(TM_NT), args, lds, s);
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string("launch of k_cpqr_team failed: ") + hipGetErrorString(e));
  return true;
}

}  // namespace spaqr
