// HIP kernels of the spaQR engine for gfx950 (CDNA4, 64-wide wavefronts).
//
//   k_copy        gathers/scatters of dense blocks (fronts, merges, packing)
//   k_qr          blocked Householder QR of a front or an interface block:
//                 one workgroup per matrix, the current JB-column panel staged
//                 in LDS, compact-WY trailing update (Section 2.4, 2.6)
//   k_scale       B <- U_i^T B R_j^{-1} on every block of the trailing matrix
//                 (block-diagonal scaling, Section 2.6)
//   k_sparsify    partial column-pivoted QR of [A_np^T | A_pn] with FP64 norms,
//                 pivots and ratio test, coarse-block write-back (Sections
//                 2.5, 2.6, and the rank rule of Section 4)
//   k_ap_*        the preconditioner apply (Section 2.8): one wavefront per
//                 front or interface, FP64 vectors, coalesced reads of the
//                 column-major factors
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace spaqr {

namespace {

constexpr int NT = 256;  // threads of the factorization kernels (4 wavefronts)
constexpr int RBMAX = 8; // right-hand sides per apply workgroup

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Exact xor partner at offset 16 or 32 by the gfx950 lane swaps
// (v_permlane16_swap: odd 16-lane rows of the first operand with even rows of
// the second; v_permlane32_swap: upper half of the first with lower half of
// the second), vector-ALU moves instead of an LDS round trip.
template <int OFF>
__device__ __forceinline__ int swap_partner(int v) {
  static_assert(OFF == 16 || OFF == 32, "lane swaps exist for offsets 16 and 32");
  if constexpr (OFF == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((threadIdx.x & 32) ? r[0] : r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((threadIdx.x & 16) ? r[0] : r[1]);
  }
}
template <int OFF>
__device__ __forceinline__ double swap_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = swap_partner<OFF>((int)(b & 0xffffffffLL));
  const int hi = swap_partner<OFF>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// xor butterfly over the wavefront (every lane gets the same sum)
__device__ __forceinline__ double wave_sum(double v) {
  v += swap_partner<32>(v);
  v += swap_partner<16>(v);
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup; every thread gets the result.  red: >= 4 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (int)(blockDim.x >> 6);
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// dlarfg convention: beta = -sign(alpha) * ||[alpha; x]||, tau = (beta - alpha)
// / beta, v = x / (alpha - beta); tau = 0 (H = I) when x = 0.
__device__ __forceinline__ void householder(double alpha, double xnorm2, double& beta, double& tau,
                                            double& scal) {
  if (xnorm2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scal = 1.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
}

// LDS layout of the QR kernel for a panel of JB columns and m rows.
template <typename T, int JB>
struct QRLds {
  static constexpr int LDP = JB + 1;  // padded row stride: conflict-free column walks
  __host__ __device__ static size_t off_t(int m) { return align16((size_t)m * LDP * sizeof(T)); }
  __host__ __device__ static size_t off_zz(int m) { return off_t(m) + align16((size_t)JB * JB * sizeof(T)); }
  __host__ __device__ static size_t off_red(int m) { return off_zz(m) + (size_t)JB * JB * sizeof(double); }
  __host__ __device__ static size_t off_tau(int m) { return off_red(m) + 8 * sizeof(double); }
  __host__ __device__ static size_t bytes(int m) { return off_tau(m) + (size_t)JB * sizeof(double); }
};

// C[0:mp, 0:ncols] (row-major, leading dimension ldc) <- H^T C with
// H = I - V Tm V^T: V (LDS, mp x JB, row stride JB+1, explicit unit diagonal,
// zeros above it and in unused columns) and Tm (LDS, JB x JB column-major,
// upper triangular).  One thread per column of C; the panel is read as
// broadcasts from LDS and the column streams through coalesced loads.
template <typename T, int JB>
__device__ void wy_apply_left(const T* __restrict__ Vs, const T* __restrict__ Tm, int mp, T* C,
                              int64_t ldc, int ncols) {
  constexpr int LDP = JB + 1;
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
    T w[JB];
#pragma unroll
    for (int t = 0; t < JB; ++t) w[t] = T(0);
    for (int r = 0; r < mp; ++r) {
      const T a = C[(int64_t)r * ldc + c];
#pragma unroll
      for (int t = 0; t < JB; ++t) w[t] += Vs[r * LDP + t] * a;
    }
    T u[JB];
#pragma unroll
    for (int t = 0; t < JB; ++t) {
      T s = T(0);
#pragma unroll
      for (int q = 0; q <= t; ++q) s += Tm[q + t * JB] * w[q];
      u[t] = s;
    }
    for (int r = 0; r < mp; ++r) {
      T s = T(0);
#pragma unroll
      for (int t = 0; t < JB; ++t) s += Vs[r * LDP + t] * u[t];
      C[(int64_t)r * ldc + c] -= s;
    }
  }
}

// Householder factorization of the LDS panel Ps (mp x jb, row stride JB+1).
// Leaves R on/above the diagonal and V below it; taus[0..jb) in LDS.
template <typename T, int JB>
__device__ bool factor_panel(T* Ps, int mp, int jb, double* taus, double* red) {
  constexpr int LDP = JB + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = (int)(blockDim.x >> 6);
  bool zero_diag = false;
  for (int t = 0; t < jb; ++t) {
    double s = 0.0;
    for (int r = t + 1 + tid; r < mp; r += blockDim.x) {
      const double v = (double)Ps[r * LDP + t];
      s += v * v;
    }
    s = block_sum(s, red);
    const double alpha = (double)Ps[t * LDP + t];
    double beta, tau, scal;
    householder(alpha, s, beta, tau, scal);
    for (int r = t + 1 + tid; r < mp; r += blockDim.x) Ps[r * LDP + t] = (T)((double)Ps[r * LDP + t] * scal);
    __syncthreads();
    for (int c = t + 1 + wv; c < jb; c += nw) {
      double acc = 0.0;
      for (int r = t + 1 + lane; r < mp; r += 64) acc += (double)Ps[r * LDP + t] * (double)Ps[r * LDP + c];
      acc = wave_sum(acc);
      const double tw = tau * (acc + (double)Ps[t * LDP + c]);
      for (int r = t + 1 + lane; r < mp; r += 64)
        Ps[r * LDP + c] = (T)((double)Ps[r * LDP + c] - tw * (double)Ps[r * LDP + t]);
      if (lane == 0) Ps[t * LDP + c] = (T)((double)Ps[t * LDP + c] - tw);
    }
    __syncthreads();
    if (tid == 0) {
      Ps[t * LDP + t] = (T)beta;
      taus[t] = tau;
    }
    if ((T)beta == T(0)) zero_diag = true;
    __syncthreads();
  }
  return zero_diag;
}

// Tm = compact-WY factor of the explicit panel V (LDS) and taus:
// T[0:t, t] = -tau_t T[0:t, 0:t] (V[:, 0:t]^T v_t), T[t, t] = tau_t.
template <typename T, int JB>
__device__ void form_t(const T* Ps, int mp, int jb, const double* taus, double* zz, T* Tm) {
  constexpr int LDP = JB + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = (int)(blockDim.x >> 6);
  for (int pidx = wv; pidx < jb * jb; pidx += nw) {
    const int i = pidx % jb, t = pidx / jb;
    if (i >= t) continue;
    double acc = 0.0;
    for (int r = t + lane; r < mp; r += 64) acc += (double)Ps[r * LDP + i] * (double)Ps[r * LDP + t];
    acc = wave_sum(acc);
    if (lane == 0) zz[i + t * JB] = acc;
  }
  for (int q = tid; q < JB * JB; q += blockDim.x) Tm[q] = T(0);
  __syncthreads();
  for (int t = 0; t < jb; ++t) {
    if (tid < t) {
      double s = 0.0;
      for (int q = tid; q < t; ++q) s += (double)Tm[tid + q * JB] * zz[q + t * JB];
      Tm[tid + t * JB] = (T)(-taus[t] * s);
    } else if (tid == t) {
      Tm[t + t * JB] = (T)taus[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- kernels
// Plain copies.  A tile is walked as one flat sequence of rows x
// cols elements so that no lane idles on short rows, with 16-byte accesses
// whenever the row length, both strides and both addresses allow them.
template <typename T>
struct Wide16;
template <>
struct Wide16<float> {
  using type = float4;
  static constexpr int N = 4;
};
template <>
struct Wide16<double> {
  using type = double2;
  static constexpr int N = 2;
};

// rows x cols elements (row strides lds, ldd) by NTH threads (thread t of
// them): element e of the tile goes to thread e mod NTH, its row and column
// advanced incrementally; src == nullptr writes zeros
template <int NTH, typename E>
__device__ __forceinline__ void copy_tile(const E* __restrict__ src, E* __restrict__ dst, int rows, int cols,
                                          int64_t lds, int64_t ldd, int t) {
  const int dr = NTH / cols, dq = NTH - dr * cols;
  int r = t / cols, q = t - r * cols;
  auto next = [&]() {
    q += dq;
    r += dr;
    if (q >= cols) {
      q -= cols;
      ++r;
    }
  };
  if (src) {
    // four elements in flight per thread (the first always in range)
    while (r < rows) {
      const int r0 = r, q0 = q;
      next();
      const int r1 = r, q1 = q;
      next();
      const int r2 = r, q2 = q;
      next();
      const int r3 = r, q3 = q;
      next();
      const E v0 = src[(int64_t)r0 * lds + q0];
      E v1{}, v2{}, v3{};
      if (r1 < rows) v1 = src[(int64_t)r1 * lds + q1];
      if (r2 < rows) v2 = src[(int64_t)r2 * lds + q2];
      if (r3 < rows) v3 = src[(int64_t)r3 * lds + q3];
      dst[(int64_t)r0 * ldd + q0] = v0;
      if (r1 < rows) dst[(int64_t)r1 * ldd + q1] = v1;
      if (r2 < rows) dst[(int64_t)r2 * ldd + q2] = v2;
      if (r3 < rows) dst[(int64_t)r3 * ldd + q3] = v3;
    }
  } else {
    for (; r < rows; next()) dst[(int64_t)r * ldd + q] = E{};
  }
}

template <int NTH, typename T>
__device__ __forceinline__ void copy_tile_any(const CopyTile<T> c, int t) {
  using W = Wide16<T>;
  constexpr int N = W::N;
  const bool wide = c.cols % N == 0 && c.ldd % N == 0 && (reinterpret_cast<uintptr_t>(c.dst) & 15) == 0 &&
                    (!c.src || (c.lds % N == 0 && (reinterpret_cast<uintptr_t>(c.src) & 15) == 0));
  if (wide)
    copy_tile<NTH>(reinterpret_cast<const typename W::type*>(c.src), reinterpret_cast<typename W::type*>(c.dst),
                   c.rows, c.cols / N, c.lds / N, c.ldd / N, t);
  else
    copy_tile<NTH>(c.src, c.dst, c.rows, c.cols, c.lds, c.ldd, t);
}

// Tiles kCopyTiles at a time per workgroup: a tile of at most
// kCopySmallBytes is copied by one wavefront, a larger one by the whole
// workgroup (no barrier is needed: the tiles of a launch never overlap).
constexpr int kCopyTiles = NT / 64;
constexpr int kCopySmallBytes = 16384;

template <typename T>
__global__ void __launch_bounds__(NT) k_copy(const CopyTile<T>* __restrict__ tiles, int64_t n) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kCopyTiles;
  const int64_t mine = t0 + wv;
  if (mine < n) {
    const CopyTile<T> c = tiles[mine];
    if (c.rows > 0 && c.cols > 0 && (int64_t)c.rows * c.cols * (int64_t)sizeof(T) <= kCopySmallBytes)
      copy_tile_any<64>(c, lane);
  }
  for (int w = 0; w < kCopyTiles && t0 + w < n; ++w) {
    const CopyTile<T> c = tiles[t0 + w];
    if (c.rows > 0 && c.cols > 0 && (int64_t)c.rows * c.cols * (int64_t)sizeof(T) > kCopySmallBytes)
      copy_tile_any<NT>(c, (int)threadIdx.x);
  }
}

// Transposing copies (row-major source, column-major destination),
// one workgroup per tile, through a 64 x 65 LDS tile: each wavefront reads
// every fourth row of a 64 x 64 sub-tile (contiguous along the row) and then
// writes every fourth column (contiguous along the column).
template <typename T>
__global__ void __launch_bounds__(NT) k_copy_t(const CopyTile<T>* __restrict__ tiles) {
  const CopyTile<T> c = tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ T t[64 * 65];
  for (int r0 = 0; r0 < c.rows; r0 += 64) {
    const int nr = min(64, c.rows - r0);
    for (int c0 = 0; c0 < c.cols; c0 += 64) {
      const int ncb = min(64, c.cols - c0);
      const T* sb = c.src + (int64_t)r0 * c.lds + c0;
      if (lane < ncb)
        for (int r = wv; r < nr; r += 4) t[lane * 65 + r] = sb[(int64_t)r * c.lds + lane];
      __syncthreads();
      T* db = c.dst + (int64_t)c0 * c.ldd + r0;
      if (lane < nr)
        for (int cc = wv; cc < ncb; cc += 4) db[(int64_t)cc * c.ldd + lane] = t[cc * 65 + lane];
      __syncthreads();
    }
  }
}

// Zero fills of several buffers in one launch; each descriptor owns the
// workgroups block0 .. block0 + ceil(words / kZeroWordsPerBlock) - 1.
__global__ void __launch_bounds__(256) k_zero(const ZeroDesc* __restrict__ ds, int64_t n) {
  int64_t lo = 0, hi = n - 1;
  const int64_t b = blockIdx.x;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ds[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const ZeroDesc d = ds[lo];
  const int64_t w0 = (b - d.block0) * kZeroWordsPerBlock;
  const int64_t w1 = min(d.words, w0 + kZeroWordsPerBlock);
  for (int64_t w = w0 + threadIdx.x; w < w1; w += 256) d.p[w] = 0u;
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
__global__ void k_scatter_nz(T* pool, const int64_t* __restrict__ dst, const double* __restrict__ val,
                             int64_t nnz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
    pool[dst[i]] = (T)val[i];
}

template <typename T, int JB>
__global__ void __launch_bounds__(NT) k_qr(const QRDesc<T>* __restrict__ descs) {
  using S = QRLds<T, JB>;
  constexpr int LDP = JB + 1;
  const QRDesc<T> d = descs[blockIdx.x];
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = d.m, n = d.n, nc = d.nc;
  const int64_t ld = d.ld ? d.ld : nc;
  T* Ps = reinterpret_cast<T*>(smem);
  T* Tm = reinterpret_cast<T*>(smem + S::off_t(m));
  double* zz = reinterpret_cast<double*>(smem + S::off_zz(m));
  double* red = reinterpret_cast<double*>(smem + S::off_red(m));
  double* taus = reinterpret_cast<double*>(smem + S::off_tau(m));
  const int tid = threadIdx.x;
  bool zero_diag = false;
  for (int j0 = 0; j0 < n; j0 += JB) {
    const int jb = min(JB, n - j0);
    const int mp = m - j0;
    T* A0 = d.a + (int64_t)j0 * ld + j0;
    for (int q = tid; q < mp * JB; q += NT) {
      const int r = q / JB, t = q - r * JB;
      Ps[r * LDP + t] = t < jb ? A0[(int64_t)r * ld + t] : T(0);
    }
    __syncthreads();
    zero_diag |= factor_panel<T, JB>(Ps, mp, jb, taus, red);
    for (int q = tid; q < mp * jb; q += NT) {
      const int r = q / jb, t = q - r * jb;
      A0[(int64_t)r * ld + t] = Ps[r * LDP + t];
    }
    if (tid < jb) d.tau[j0 + tid] = (T)taus[tid];
    __syncthreads();
    for (int q = tid; q < mp * jb; q += NT) {
      const int r = q / jb, t = q - r * jb;
      if (r < t) Ps[r * LDP + t] = T(0);
      else if (r == t) Ps[r * LDP + t] = T(1);
    }
    __syncthreads();
    form_t<T, JB>(Ps, mp, jb, taus, zz, Tm);
    if (d.tpan)
      for (int q = tid; q < JB * JB; q += NT) d.tpan[(int64_t)(j0 / JB) * JB * JB + q] = Tm[q];
    wy_apply_left<T, JB>(Ps, Tm, mp, A0 + jb, ld, nc - j0 - jb);
    __syncthreads();
  }
  if (tid == 0 && zero_diag && d.flag) *d.flag = 1;
}

// ------------------------------------------------ register-panel front QR
// 16-byte LDS vectors: JB consecutive values of a row in JB*sizeof(T)/16 reads.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int N = 4;
  __device__ static void put(const float4& v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
  __device__ static float4 get(const float* o) { return make_float4(o[0], o[1], o[2], o[3]); }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int N = 2;
  __device__ static void put(const double2& v, double* o) { o[0] = v.x; o[1] = v.y; }
  __device__ static double2 get(const double* o) { return make_double2(o[0], o[1]); }
};

template <typename T, int JB>
__device__ __forceinline__ void lds_load_row(const T* p, T (&out)[JB]) {
  using V = Vec16<T>;
  const typename V::type* q = reinterpret_cast<const typename V::type*>(p);
#pragma unroll
  for (int i = 0; i < JB / V::N; ++i) V::put(q[i], out + i * V::N);
}

template <typename T, int JB>
__device__ __forceinline__ void lds_store_row(T* p, const T (&in)[JB]) {
  using V = Vec16<T>;
  typename V::type* q = reinterpret_cast<typename V::type*>(p);
#pragma unroll
  for (int i = 0; i < JB / V::N; ++i) q[i] = V::get(in + i * V::N);
}

// acc += s * row, row read as 16-byte vectors
template <typename T, int JB>
__device__ __forceinline__ void lds_axpy_row(const T* p, T s, T (&acc)[JB]) {
  using V = Vec16<T>;
  const typename V::type* q = reinterpret_cast<const typename V::type*>(p);
#pragma unroll
  for (int i = 0; i < JB / V::N; ++i) {
    T tmp[V::N];
    V::put(q[i], tmp);
#pragma unroll
    for (int k = 0; k < V::N; ++k) acc[i * V::N + k] += tmp[k] * s;
  }
}

// row . u, row read as 16-byte vectors
template <typename T, int JB>
__device__ __forceinline__ T lds_dot_row(const T* p, const T (&u)[JB]) {
  using V = Vec16<T>;
  const typename V::type* q = reinterpret_cast<const typename V::type*>(p);
  T s = T(0);
#pragma unroll
  for (int i = 0; i < JB / V::N; ++i) {
    T tmp[V::N];
    V::put(q[i], tmp);
#pragma unroll
    for (int k = 0; k < V::N; ++k) s += tmp[k] * u[i * V::N + k];
  }
  return s;
}

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// Compile-time loop: f(integral_constant<int, I>) for I = 0 .. N-1.  Register
// arrays indexed this way stay in registers; a runtime index would turn every
// access into a chain of compares and selects.
template <int... Is, typename F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F&& f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

// Exchange with a partner lane for the butterfly levels below.  Distances
// 16 and 32 go through ds_bpermute; the shorter ones use DPP lane moves
// inside a row of 16 lanes: row_mirror (lane i <-> 15 - i) pairs lanes that
// differ in bit 3, row_half_mirror (i <-> 7 - i) lanes that differ in bit 2,
// quad_perm swaps bit 1 or bit 0.  Each pairing flips exactly the level's own
// bit among the bits not yet reduced, which is all a butterfly needs.
template <int OFF>
__device__ __forceinline__ int dpp_partner(int v) {
  constexpr int CTRL = OFF == 8 ? 0x140 : (OFF == 4 ? 0x141 : (OFF == 2 ? 0x4E : 0xB1));
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int OFF, typename T>
__device__ __forceinline__ T xshfl(T v) {
  if constexpr (OFF >= 16) {
    if constexpr (std::is_same<T, int>::value) {
      return swap_partner<OFF>(v);
    } else if constexpr (sizeof(T) == 4) {
      return __int_as_float(swap_partner<OFF>(__float_as_int(v)));
    } else {
      return swap_partner<OFF>((double)v);
    }
  } else if constexpr (std::is_same<T, int>::value) {
    return dpp_partner<OFF>(v);
  } else if constexpr (sizeof(T) == 4) {
    return __int_as_float(dpp_partner<OFF>(__float_as_int(v)));
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_partner<OFF>((int)(b & 0xffffffffLL));
    const int hi = dpp_partner<OFF>((int)(b >> 32));
    return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
  }
}

// Reduce-scatter of H2 = 2 H per-lane values over the wavefront, one
// butterfly level per call: lanes with bit OFF set keep the upper half.
template <typename T, int H, int OFF, int JB>
__device__ __forceinline__ void rs_level(T (&v)[JB], int lane) {
  if constexpr (H >= 1) {
    const bool hi = (lane & OFF) != 0;
    sfor<H>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const T lo_v = v[i], hi_v = v[i + H];
      const T send = hi ? lo_v : hi_v;
      const T keep = hi ? hi_v : lo_v;
      v[i] = keep + xshfl<OFF>(send);
    });
    rs_level<T, H / 2, OFF / 2, JB>(v, lane);
  }
}

// On return every lane holds the wave total of value index
// lane >> (6 - log2 JB).  JB values cost JB - 1 + (6 - log2 JB) shuffles
// instead of 6 JB.
template <typename T, int JB>
__device__ __forceinline__ T wave_reduce_scatter(T (&v)[JB]) {
  const int lane = threadIdx.x & 63;
  rs_level<T, JB / 2, 32, JB>(v, lane);
  T s = v[0];
  constexpr int OFF0 = 32 >> ilog2c(JB);
  if constexpr (OFF0 >= 8) s += xshfl<8>(s);
  if constexpr (OFF0 >= 4) s += xshfl<4>(s);
  if constexpr (OFF0 >= 2) s += xshfl<2>(s);
  s += xshfl<1>(s);
  return s;
}

// Blocked Householder QR of one front (row-major m x nc, the first n columns
// pivots), panels of JB columns held in registers: thread tid owns panel rows
// tid + NT q, q < Q, so m <= NT Q.  For column t of a panel one workgroup
// reduction yields the whole row t of the Gram matrix of the rows below t:
// the tail norm (Householder vector, dlarfg convention), the dots with the
// later panel columns (their update) and the dots with the earlier
// reflectors (column t of the compact-WY factor T).  One barrier per column.
// The trailing columns are then updated as C <- C - V T^T (V^T C), one thread
// per column, V read from LDS as aligned vectors.  Outputs as k_qr: R and V
// in place, tau, T panels (column-major, JB x JB per panel) and the
// zero-diagonal flag.
template <typename T, int JB, int Q>
__global__ void __launch_bounds__(NT) k_qr_reg(const QRDesc<T>* __restrict__ descs) {
  constexpr int SH = 6 - ilog2c(JB);
  const QRDesc<T> d = descs[blockIdx.x];
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = d.m, n = d.n, nc = d.nc, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t ld = d.ld ? d.ld : nc;
  T* Vs = reinterpret_cast<T*>(smem);  // m x JB row-major, explicit unit diagonal
  T* Ts = Vs + (size_t)m * JB;         // JB x JB, row i of T at i * JB
  T* red = Ts + JB * JB;               // 2 buffers x 4 waves x JB
  T* rowt = red + 8 * JB;              // 2 buffers x JB
  bool zero_diag = false;
  for (int j0 = 0; j0 < n; j0 += JB) {
    const int jb = min(JB, n - j0), mp = m - j0;
    T* A0 = d.a + (int64_t)j0 * ld + j0;
    T a[Q][JB];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = tid + NT * q;
#pragma unroll
      for (int c = 0; c < JB; ++c) a[q][c] = (r < mp && c < jb) ? A0[(int64_t)r * ld + c] : T(0);
    }
    T trow[JB];
#pragma unroll
    for (int c = 0; c < JB; ++c) trow[c] = T(0);
    sfor<JB>([&](auto TC) {
      constexpr int t = decltype(TC)::value;
      if (t >= jb) return;  // uniform
      constexpr int buf = t & 1;
      T v[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) v[c] = T(0);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = tid + NT * q;
        if (r > t && r < mp) {
          const T x = a[q][t];
#pragma unroll
          for (int c = 0; c < JB; ++c) v[c] += x * a[q][c];
        }
      }
      if (tid == t) lds_store_row<T, JB>(rowt + buf * JB, a[0]);
      const T s = wave_reduce_scatter<T, JB>(v);
      if ((lane & ((1 << SH) - 1)) == 0) red[(buf * 4 + wv) * JB + (lane >> SH)] = s;
      __syncthreads();
      T g[JB], at[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) g[c] = T(0);
#pragma unroll
      for (int w = 0; w < 4; ++w) lds_axpy_row<T, JB>(red + (buf * 4 + w) * JB, T(1), g);
      lds_load_row<T, JB>(rowt + buf * JB, at);
      double beta, tau, scal;
      householder((double)at[t], (double)g[t], beta, tau, scal);
      const T sc = (T)scal, ta = (T)tau;
      // z_c = v_c . v_t for c < t (T column), coef_c = tau v_t . a_c for c > t
      T z[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) z[c] = at[c] + sc * g[c];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int r = tid + NT * q;
        if (r > t && r < mp) {
          const T x = a[q][t] * sc;
          a[q][t] = x;
#pragma unroll
          for (int c = t + 1; c < JB; ++c) a[q][c] -= (ta * z[c]) * x;
        }
      }
      if (tid == t) {
        a[0][t] = (T)beta;
#pragma unroll
        for (int c = t + 1; c < JB; ++c) a[0][c] -= ta * z[c];
        d.tau[j0 + t] = ta;
        trow[t] = ta;
      }
      if (tid < t) {
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < t; ++c) acc += trow[c] * z[c];
        trow[t] = -ta * acc;
      }
      if ((T)beta == T(0)) zero_diag = true;
    });
    // R and V back to the front, explicit V and T to LDS, T panel out
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = tid + NT * q;
      if (r < mp) {
        T vrow[JB];
#pragma unroll
        for (int c = 0; c < JB; ++c) {
          if (c < jb) A0[(int64_t)r * ld + c] = a[q][c];
          vrow[c] = c >= jb ? T(0) : (r > c ? a[q][c] : (r == c ? T(1) : T(0)));
        }
        lds_store_row<T, JB>(Vs + (size_t)r * JB, vrow);
      }
    }
    if (tid < JB) {
      lds_store_row<T, JB>(Ts + tid * JB, trow);
      if (d.tpan) {
        T* tp = d.tpan + (int64_t)(j0 / JB) * JB * JB;
#pragma unroll
        for (int c = 0; c < JB; ++c) tp[tid + c * JB] = trow[c];
      }
    }
    __syncthreads();
    // trailing columns: C <- C - V (T^T (V^T C)); four adjacent lanes share a
    // column, lane part p taking rows p, p + 4, ...
    const int ncols = nc - j0 - jb, part = tid & 3;
    for (int cb = tid >> 2; cb < ((ncols + 15) & ~15); cb += NT / 4) {
      const bool live = cb < ncols;
      T* Cc = A0 + jb + (live ? cb : 0);
      T w[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) w[c] = T(0);
      if (live) {
        int r = part;
        for (; r + 28 < mp; r += 32) {
          T cv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) cv[e] = Cc[(int64_t)(r + 4 * e) * ld];
#pragma unroll
          for (int e = 0; e < 8; ++e) lds_axpy_row<T, JB>(Vs + (size_t)(r + 4 * e) * JB, cv[e], w);
        }
        for (; r < mp; r += 4) lds_axpy_row<T, JB>(Vs + (size_t)r * JB, Cc[(int64_t)r * ld], w);
      }
#pragma unroll
      for (int c = 0; c < JB; ++c) {
        w[c] += xshfl<1>(w[c]);
        w[c] += xshfl<2>(w[c]);
      }
      if (!live) continue;
      T u[JB];
#pragma unroll
      for (int c = 0; c < JB; ++c) u[c] = T(0);
#pragma unroll
      for (int q = 0; q < JB; ++q) lds_axpy_row<T, JB>(Ts + q * JB, w[q], u);
      int r = part;
      for (; r + 28 < mp; r += 32) {
        T cv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) cv[e] = Cc[(int64_t)(r + 4 * e) * ld];
#pragma unroll
        for (int e = 0; e < 8; ++e)
          Cc[(int64_t)(r + 4 * e) * ld] = cv[e] - lds_dot_row<T, JB>(Vs + (size_t)(r + 4 * e) * JB, u);
      }
      for (; r < mp; r += 4) Cc[(int64_t)r * ld] -= lds_dot_row<T, JB>(Vs + (size_t)r * JB, u);
    }
    __syncthreads();
  }
  if (tid == 0 && zero_diag && d.flag) *d.flag = 1;
}

// Trailing update of a column slice of a front (TrailDesc): the slice
// (m x CW) stays in LDS while every JB-reflector panel of the pivot block is
// applied, C <- C - V T^T (V^T C).  Thread (c, g) = (tid % CW, tid / CW) owns
// slice column c and rows g, g + TY, ...; V rows are read from the factored
// pivot block (row stride a multiple of the vector width) and shared by the
// CW lanes of a row group.  Per panel: partial V^T C over the row groups,
// one LDS reduction, T^T W by JB row-group lanes, then the update.
template <typename T, int JB, int CW>
__global__ void __launch_bounds__(NT) k_trail(const TrailDesc<T>* __restrict__ ds) {
  constexpr int TY = NT / CW;
  static_assert(TY >= JB, "row groups must cover the panel width");
  using V = Vec16<T>;
  const TrailDesc<T> d = ds[blockIdx.x];
  if (d.flag && *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* red = reinterpret_cast<T*>(smem);     // TY x JB x CW partials
  T* Ws = red + TY * JB * CW;              // JB x CW
  T* Us = Ws + JB * CW;                    // JB x CW
  T* Cs = Us + JB * CW;                    // m x (CW + 1)
  constexpr int LC = CW + 1;
  const int tid = threadIdx.x, c = tid % CW, g = tid / CW;
  const int m = d.m, n = d.n;
  const int64_t ld = d.ld, ldc = d.ldc;
  const bool live = c < d.cw;
  T* col = d.c + d.c0 + c;
  for (int r = g; r < m; r += TY) Cs[r * LC + c] = live ? col[(int64_t)r * ldc] : T(0);
  __syncthreads();
  for (int p0 = 0; p0 < n; p0 += JB) {
    const int jb = min(JB, n - p0);
    const T* vp = d.a + p0;  // V of this panel: columns p0 .. p0 + jb - 1
    T w[JB];
#pragma unroll
    for (int t = 0; t < JB; ++t) w[t] = T(0);
    for (int r = p0 + g; r < m; r += TY) {
      const T x = Cs[r * LC + c];
      T v[JB];
      const typename V::type* q = reinterpret_cast<const typename V::type*>(vp + (int64_t)r * ld);
#pragma unroll
      for (int i = 0; i < JB / V::N; ++i) V::put(q[i], v + i * V::N);
      const int rr = r - p0;
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const T vt = t >= jb ? T(0) : (rr > t ? v[t] : (rr == t ? T(1) : T(0)));
        w[t] += vt * x;
      }
    }
#pragma unroll
    for (int t = 0; t < JB; ++t) red[(g * JB + t) * CW + c] = w[t];
    __syncthreads();
    if (g < JB) {
      T sum = T(0);
      for (int h = 0; h < TY; ++h) sum += red[(h * JB + g) * CW + c];
      Ws[g * CW + c] = sum;
    }
    __syncthreads();
    if (g < JB) {
      const T* tp = d.tpan + (int64_t)(p0 / JB) * JB * JB;  // T[q][g] at q + g JB
      T u = T(0);
      for (int q2 = 0; q2 <= g; ++q2) u += tp[q2 + g * JB] * Ws[q2 * CW + c];
      Us[g * CW + c] = u;
    }
    __syncthreads();
    T u[JB];
#pragma unroll
    for (int t = 0; t < JB; ++t) u[t] = Us[t * CW + c];
    for (int r = p0 + g; r < m; r += TY) {
      T v[JB];
      const typename V::type* q = reinterpret_cast<const typename V::type*>(vp + (int64_t)r * ld);
#pragma unroll
      for (int i = 0; i < JB / V::N; ++i) V::put(q[i], v + i * V::N);
      const int rr = r - p0;
      T acc = T(0);
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const T vt = t >= jb ? T(0) : (rr > t ? v[t] : (rr == t ? T(1) : T(0)));
        acc += vt * u[t];
      }
      Cs[r * LC + c] -= acc;
    }
    __syncthreads();
  }
  if (live)
    for (int r = g; r < m; r += TY) col[(int64_t)r * ldc] = Cs[r * LC + c];
}

// ------------------------------------------------------------------------
// Blocked WY trailing update on the matrix cores (Section 2.4: H_s^T applied
// to the trailing columns of a front, or U_pp^T to the blocks right of a
// scaled interface).  The reflectors of a factored pivot block are taken 64
// at a time, H_j0 ... H_{j0+63} = I - V_b T_b V_b^T, and every 64-column tile
// C of the trailing matrix gets C <- C - V_b (T_b^T (V_b^T C)): two
// contractions over the rows, on FP32 (or FP64) MFMA 16x16x4 tiles with
// accumulation in the same precision.
//
// One 16x16x4 MFMA multiplies A (16 x 4) by B (4 x 16) into D (16 x 16); lane
// l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Accumulator v of lane l
// holds D[row(l / 16, v)][l % 16]: row 4 (l / 16) + v for FP32, row
// l / 16 + 4 v for FP64 (the two instructions distribute D's rows
// differently, as measured on gfx950).
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  typedef float acc __attribute__((ext_vector_type(4)));
  __device__ static acc mma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int kk, int v) { return 4 * kk + v; }
};
template <>
struct Mfma16<double> {
  typedef double acc __attribute__((ext_vector_type(4)));
  __device__ static acc mma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int kk, int v) { return kk + 4 * v; }
};

constexpr int WYB = 64;  // reflectors per block, columns per tile

// v_i(r) of the factored pivot block: explicit below the diagonal, the unit
// diagonal and the zeros above it implied (i = reflector index, global)
template <typename T>
__device__ __forceinline__ T wy_v(const T* a, int64_t ld, int m, int nref, int r, int i) {
  if (i >= nref || r >= m || r < i) return T(0);
  return r == i ? T(1) : a[(int64_t)r * ld + i];
}

// T_b of one block of 64 reflectors from G = V_b^T V_b and tau: T[i][i] =
// tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i] (the forward, columnwise
// compact-WY recurrence).  One workgroup (4 waves) per block: wave w forms
// rows 16 w .. 16 w + 15 of G on the matrix cores; wave 0 then runs the
// recurrence in LDS.  T_b is written row-major 64 x 64, zero outside the
// upper triangle of the block's nb reflectors.
template <typename T>
__global__ void __launch_bounds__(256) k_wy_tblock(const WYBlock<T>* __restrict__ ds) {
  using M = Mfma16<T>;
  const WYBlock<T> d = ds[blockIdx.x];
  __shared__ T G[WYB][WYB + 1];
  __shared__ T Tm[WYB][WYB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j0 = d.j0, nref = d.n, m = d.m;
  const int64_t ld = d.ld;
  const int nb = min(WYB, nref - j0);
  const int kk = lane >> 4, ii = lane & 15;
  typename M::acc acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = typename M::acc{0, 0, 0, 0};
  for (int r = j0; r < m; r += 16) {
    T av[4], bv[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int rr = r + 4 * u + kk;
      av[u] = wy_v(d.a, ld, m, j0 + nb, rr, j0 + 16 * wv + ii);
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[u][t] = wy_v(d.a, ld, m, j0 + nb, rr, j0 + 16 * t + ii);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = M::mma(av[u], bv[u][t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) G[16 * wv + M::row(kk, v)][16 * t + ii] = acc[t][v];
  for (int q = tid; q < WYB * WYB; q += 256) Tm[q / WYB][q % WYB] = T(0);
  __syncthreads();
  if (wv == 0) {
    // column i of T: lane j < i forms T[j][i] from its own row of T
    for (int i = 0; i < nb; ++i) {
      const T tau_i = d.tau[j0 + i];
      T y = T(0);
      if (lane < i)
        for (int q = lane; q < i; ++q) y += Tm[lane][q] * G[q][i];
      // lane j reads and writes row j of T only: no exchange between lanes
      if (lane < i) Tm[lane][i] = -tau_i * y;
      if (lane == i) Tm[i][i] = tau_i;
    }
  }
  __syncthreads();
  T* out = d.tblk;
  for (int q = tid; q < WYB * WYB; q += 256) out[q] = Tm[q / WYB][q % WYB];
}

// C <- H_0^T ... H_{n-1}^T C on one tile of at most 64 trailing columns
// (WYTile), block by block: W = V_b^T C (64 x 64), U = T_b^T W, C -= V_b U.
// Wave w forms rows 16 w .. 16 w + 15 of W and U; the update runs over
// 16-row chunks of C, chunk q on wave q % 4.  C is re-read from memory for
// every block (the tile is 64 columns by all the front's rows).
template <typename T>
__global__ void __launch_bounds__(256) k_trail_mfma(const WYTile<T>* __restrict__ ds) {
  using M = Mfma16<T>;
  const WYTile<T> d = ds[blockIdx.x];
  if (d.flag && *d.flag != 0) return;
  __shared__ T Ws[WYB][WYB + 1];
  __shared__ T Us[WYB][WYB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int kk = lane >> 4, ii = lane & 15;
  const int m = d.m, nref = d.n, cw = d.cw;
  const int64_t ld = d.ld, ldc = d.ldc;
  T* C = d.c + d.c0;
  auto cval = [&](int r, int c) -> T { return (r < m && c < cw) ? C[(int64_t)r * ldc + c] : T(0); };
  for (int j0 = 0, b = 0; j0 < nref; j0 += WYB, ++b) {
    const int jend = min(nref, j0 + WYB);
    // W = V_b^T C over rows j0 .. m - 1
    typename M::acc acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = typename M::acc{0, 0, 0, 0};
    for (int r = j0; r < m; r += 16) {
      T av[4], bv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int rr = r + 4 * u + kk;
        av[u] = wy_v(d.a, ld, m, jend, rr, j0 + 16 * wv + ii);
#pragma unroll
        for (int t = 0; t < 4; ++t) bv[u][t] = cval(rr, 16 * t + ii);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = M::mma(av[u], bv[u][t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Ws[16 * wv + M::row(kk, v)][16 * t + ii] = acc[t][v];
    __syncthreads();
    // U = T_b^T W (T_b row-major 64 x 64, upper triangular)
    const T* Tb = d.tblk + (int64_t)b * WYB * WYB;
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = typename M::acc{0, 0, 0, 0};
    for (int q = 0; q < WYB; q += 4) {
      const T a = Tb[(q + kk) * WYB + 16 * wv + ii];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = M::mma(a, Ws[q + kk][16 * t + ii], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) Us[16 * wv + M::row(kk, v)][16 * t + ii] = acc[t][v];
    __syncthreads();
    // C -= V_b U on 16-row chunks
    for (int r0 = j0 + 16 * wv; r0 < m; r0 += 64) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] = cval(r0 + M::row(kk, v), 16 * t + ii);
      for (int q = 0; q < WYB; q += 4) {
        const T a = -wy_v(d.a, ld, m, jend, r0 + ii, j0 + q + kk);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = M::mma(a, Us[q + kk][16 * t + ii], acc[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = r0 + M::row(kk, v), c = 16 * t + ii;
          if (r < m && c < cw) C[(int64_t)r * ldc + c] = acc[t][v];
        }
    }
    __syncthreads();
  }
}

// Scaling of the blocks touching an interface (Algorithm 2, scaling step):
// B <- Q_i^T B for the block's row interface i.  Workgroup (block, y) owns
// the block's columns y NT .. y NT + NT - 1; the compact-WY panels of Q_i
// are staged in LDS one at a time.  A diagonal block becomes the identity.
template <typename T, int JB>
__global__ void __launch_bounds__(NT) k_scale(const ScaleBlk<T>* __restrict__ descs,
                                              const ScaleFac<T>* __restrict__ fac) {
  using S = QRLds<T, JB>;
  constexpr int LDP = JB + 1;
  const ScaleBlk<T> d = descs[blockIdx.x];
  T* B = d.B;
  const int rows = d.rows, cols = d.cols, tid = threadIdx.x;
  const int c0 = (int)blockIdx.y * NT;
  if (c0 >= cols) return;
  const int nc = min(NT, cols - c0);
  const bool si = d.fi >= 0 && *fac[d.fi].flag == 0;
  if (d.fi >= 0 && d.fi == d.fj) {
    if (si && tid < nc)
      for (int r = 0; r < rows; ++r) B[(int64_t)r * cols + c0 + tid] = r == c0 + tid ? T(1) : T(0);
    return;
  }
  if (!si) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* Vs = reinterpret_cast<T*>(smem);
  T* Tm = reinterpret_cast<T*>(smem + S::off_t(rows));
  const ScaleFac<T> f = fac[d.fi];
  for (int j0 = 0; j0 < rows; j0 += JB) {
    const int jb = min(JB, rows - j0), mp = rows - j0;
    for (int q = tid; q < mp * JB; q += NT) {
      const int r = q / JB, t = q - r * JB;
      T v;
      if (t >= jb || r < t) v = T(0);
      else if (r == t) v = T(1);
      else v = f.vr[(int64_t)(j0 + r) + (int64_t)(j0 + t) * rows];
      Vs[r * LDP + t] = v;
    }
    for (int q = tid; q < JB * JB; q += NT) Tm[q] = f.tpan[(int64_t)(j0 / JB) * JB * JB + q];
    __syncthreads();
    wy_apply_left<T, JB>(Vs, Tm, mp, B + (int64_t)j0 * cols + c0, cols, nc);
    __syncthreads();
  }
}

// Both factors of the scaling step for a block of at most 64 x 64: the block
// is loaded into LDS once, Q_i^T applied panel by panel (W = V^T B and
// B -= V (T^T W), all products spread over the workgroup), then B R_j^{-1}
// by forward substitution along each row (R_j staged in LDS), and the block
// written back once.
template <typename T, int JB>
__global__ void __launch_bounds__(NT) k_scale_small(const ScaleBlk<T>* __restrict__ descs,
                                                    const ScaleFac<T>* __restrict__ fac, int max_rows,
                                                    int max_cols) {
  const ScaleBlk<T> d = descs[blockIdx.x];
  T* B = d.B;
  const int rows = d.rows, cols = d.cols, tid = threadIdx.x;
  const bool si = d.fi >= 0 && *fac[d.fi].flag == 0;
  if (d.fi >= 0 && d.fi == d.fj) {
    if (si)
      for (int q = tid; q < rows * cols; q += NT) {
        const int r = q / cols, c = q - r * cols;
        B[q] = r == c ? T(1) : T(0);
      }
    return;
  }
  const bool sj = d.fj >= 0 && *fac[d.fj].flag == 0;
  if (!si && !sj) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int LB = max_cols + 1;
  T* Bs = reinterpret_cast<T*>(smem);                 // max_rows x LB
  T* Vs = Bs + (size_t)max_rows * LB;                 // max_rows x (JB + 1)
  T* Tm = Vs + (size_t)max_rows * (JB + 1);           // JB x JB
  T* W = Tm + JB * JB;                                // JB x max_cols
  T* U = W + (size_t)JB * max_cols;                   // JB x max_cols
  T* Rs = W;  // max_cols x LB, over W and U: the left factor is done with them by then
  for (int q = tid; q < rows * cols; q += NT) {
    const int r = q / cols, c = q - r * cols;
    Bs[r * LB + c] = B[q];
  }
  if (si) {
    const ScaleFac<T> f = fac[d.fi];
    for (int j0 = 0; j0 < rows; j0 += JB) {
      const int jb = min(JB, rows - j0), mp = rows - j0;
      for (int q = tid; q < mp * JB; q += NT) {
        const int r = q / JB, t = q - r * JB;
        T v;
        if (t >= jb || r < t) v = T(0);
        else if (r == t) v = T(1);
        else v = f.vr[(int64_t)(j0 + r) + (int64_t)(j0 + t) * rows];
        Vs[r * (JB + 1) + t] = v;
      }
      for (int q = tid; q < JB * JB; q += NT) Tm[q] = f.tpan[(int64_t)(j0 / JB) * JB * JB + q];
      __syncthreads();
      for (int q = tid; q < JB * cols; q += NT) {
        const int t = q / cols, c = q - t * cols;
        T w = T(0);
        for (int r = 0; r < mp; ++r) w += Vs[r * (JB + 1) + t] * Bs[(j0 + r) * LB + c];
        W[t * max_cols + c] = w;
      }
      __syncthreads();
      for (int q = tid; q < JB * cols; q += NT) {
        const int t = q / cols, c = q - t * cols;
        T u = T(0);
        for (int q2 = 0; q2 <= t; ++q2) u += Tm[q2 + t * JB] * W[q2 * max_cols + c];
        U[t * max_cols + c] = u;
      }
      __syncthreads();
      for (int q = tid; q < mp * cols; q += NT) {
        const int r = q / cols, c = q - r * cols;
        T acc = T(0);
#pragma unroll
        for (int t = 0; t < JB; ++t) acc += Vs[r * (JB + 1) + t] * U[t * max_cols + c];
        Bs[(j0 + r) * LB + c] -= acc;
      }
      __syncthreads();
    }
  }
  if (sj) {
    const T* R = fac[d.fj].vr;  // R[q][c] at q + c cols
    for (int q = tid; q < cols * cols; q += NT) {
      const int c = q / cols, r = q - c * cols;
      Rs[r * LB + c] = R[q];
    }
    __syncthreads();
    // column panels of 16: the panel's entries are first reduced by the
    // solved columns to their left (all rows x 16 entries in parallel), then
    // each row solves the panel's 16 x 16 triangle
    for (int p0 = 0; p0 < cols; p0 += 16) {
      const int pw = min(16, cols - p0);
      if (p0 > 0)
        for (int q = tid; q < rows * pw; q += NT) {
          const int r = q / pw, c = p0 + (q - r * pw);
          T x = Bs[r * LB + c];
          for (int q2 = 0; q2 < p0; ++q2) x -= Bs[r * LB + q2] * Rs[q2 * LB + c];
          Bs[r * LB + c] = x;
        }
      __syncthreads();
      for (int r = tid; r < rows; r += NT)
        for (int c = p0; c < p0 + pw; ++c) {
          T x = Bs[r * LB + c];
          for (int q2 = p0; q2 < c; ++q2) x -= Bs[r * LB + q2] * Rs[q2 * LB + c];
          Bs[r * LB + c] = x / Rs[c * LB + c];
        }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int q = tid; q < rows * cols; q += NT) {
    const int r = q / cols, c = q - r * cols;
    B[q] = Bs[r * LB + c];
  }
}

// B <- B R_j^{-1} for the block's column interface j (the right factor of the
// scaling step), R_j upper triangular with R[q][c] at q + c cols.  Workgroup
// (block, y) owns rows 16 y .. 16 y + 15.  Columns go in panels of 16: a
// panel is first reduced by the solved columns to its left (tiles of 64
// through LDS, one output per thread), then solved against the panel's
// diagonal block by forward substitution, one row per thread.
template <typename T>
__global__ void __launch_bounds__(NT) k_scale_right(const ScaleBlk<T>* __restrict__ descs,
                                                    const ScaleFac<T>* __restrict__ fac) {
  constexpr int RB = 16, NB = 16, KC = 64;
  static_assert(RB * NB == NT, "one output per thread");
  const ScaleBlk<T> d = descs[blockIdx.x];
  if (d.fj < 0 || d.fi == d.fj || *fac[d.fj].flag != 0) return;
  const int rows = d.rows, cols = d.cols, r0 = (int)blockIdx.y * RB;
  if (r0 >= rows) return;
  const int rb = min(RB, rows - r0);
  const T* R = fac[d.fj].vr;
  T* B = d.B + (int64_t)r0 * cols;
  __shared__ T Xs[RB][KC + 1];
  __shared__ T Rs[KC][NB + 1];
  __shared__ T Ps[RB][NB + 1];
  __shared__ T Rt[NB][NB + 1];
  const int tid = threadIdx.x, i = tid / NB, cc = tid - i * NB;
  for (int p0 = 0; p0 < cols; p0 += NB) {
    const int nb = min(NB, cols - p0);
    T acc = T(0);
    for (int q0 = 0; q0 < p0; q0 += KC) {
      const int kq = min(KC, p0 - q0);
      for (int e = tid; e < RB * KC; e += NT) {
        const int ii = e / KC, k = e - ii * KC;
        Xs[ii][k] = (ii < rb && k < kq) ? B[(int64_t)ii * cols + q0 + k] : T(0);
      }
      for (int e = tid; e < KC * NB; e += NT) {
        const int c = e / KC, k = e - c * KC;
        Rs[k][c] = (c < nb && k < kq) ? R[(int64_t)(q0 + k) + (int64_t)(p0 + c) * cols] : T(0);
      }
      __syncthreads();
#pragma unroll 16
      for (int k = 0; k < KC; ++k) acc += Xs[i][k] * Rs[k][cc];
      __syncthreads();
    }
    Ps[i][cc] = (i < rb && cc < nb) ? B[(int64_t)i * cols + p0 + cc] - acc : T(0);
    Rt[i][cc] = (i < nb && cc < nb) ? R[(int64_t)(p0 + i) + (int64_t)(p0 + cc) * cols] : T(0);
    __syncthreads();
    if (tid < rb)
      for (int c = 0; c < nb; ++c) {
        T x = Ps[tid][c];
        for (int q = 0; q < c; ++q) x -= Ps[tid][q] * Rt[q][c];
        Ps[tid][c] = x / Rt[c][c];
      }
    __syncthreads();
    if (i < rb && cc < nb) B[(int64_t)i * cols + p0 + cc] = Ps[i][cc];
    __syncthreads();  // the next panel reads these columns
  }
}

template <typename T>
__global__ void __launch_bounds__(NT) k_sparsify(const SpDesc<T>* __restrict__ descs,
                                                 const SpNbr* __restrict__ nbrs) {
  const SpDesc<T> d = descs[blockIdx.x];
  const double eps = d.eps;
  T* pool = d.pool;
  int* rank = d.rank;
  const int P = d.P, tid = threadIdx.x;
  if (P == 0 || *d.flag != 0) return;  // not scaled: rank stays P
  extern __shared__ __align__(16) unsigned char smem[];
  const int nnb = d.nrow + d.ncol;
  int* off = reinterpret_cast<int*>(smem);
  double* vbuf = reinterpret_cast<double*>(smem + align16((size_t)(nnb + 1) * sizeof(int)));
  double* red = vbuf + P;
  double* bv = red + 8;
  int* bi = reinterpret_cast<int*>(bv + NT);
  const SpNbr* nb = nbrs + d.nb;
  if (tid == 0) {
    int o = 0;
    for (int b = 0; b < nnb; ++b) {
      off[b] = o;
      o += rank[nb[b].cluster];
    }
    off[nnb] = o;
  }
  __syncthreads();
  const int m = off[nnb];
  const int64_t ldc = d.mmax;
  T* C = d.C;
  // C = [A_np^T | A_pn], P x m row-major
  for (int b = 0; b < nnb; ++b) {
    const int w = off[b + 1] - off[b];
    const T* blk = pool + nb[b].blk;
    const int64_t ld = nb[b].ld;
    const int o = off[b];
    if (b < d.nrow) {
      for (int e = tid; e < w * P; e += NT) {
        const int a = e / P, q = e - a * P;
        C[(int64_t)q * ldc + o + a] = blk[(int64_t)a * ld + q];
      }
    } else {
      for (int e = tid; e < w * P; e += NT) {
        const int q = e / w, a = e - q * w;
        C[(int64_t)q * ldc + o + a] = blk[(int64_t)q * ld + a];
      }
    }
  }
  __syncthreads();
  double* nrm = d.nrm;
  int* perm = d.perm;
  int* ipos = d.perm + d.mmax;
  for (int c = tid; c < m; c += NT) {
    double s = 0.0;
    for (int q = 0; q < P; ++q) {
      const double v = (double)C[(int64_t)q * ldc + c];
      s += v * v;
    }
    nrm[c] = s;
    perm[c] = c;
  }
  __syncthreads();
  const int kmax = min(P, m);
  int r = 0;
  double R11 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    // pivot: largest remaining norm, ties to the lowest position
    double best = -1.0;
    int bidx = m;
    for (int c = k + tid; c < m; c += NT) {
      const double v = nrm[c];
      if (v > best) {
        best = v;
        bidx = c;
      }
    }
    bv[tid] = best;
    bi[tid] = bidx;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
      if (tid < st) {
        const double v2 = bv[tid + st];
        const int i2 = bi[tid + st];
        if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) {
          bv[tid] = v2;
          bi[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int piv = bi[0];
    const double rkk = sqrt(bv[0]);
    __syncthreads();
    if (k == 0) {
      R11 = rkk;
      if (R11 == 0.0) break;
    }
    if (eps > 0.0 && rkk < eps * R11) break;
    if (piv != k) {
      for (int q = tid; q < P; q += NT) {
        const T a = C[(int64_t)q * ldc + k];
        C[(int64_t)q * ldc + k] = C[(int64_t)q * ldc + piv];
        C[(int64_t)q * ldc + piv] = a;
      }
      if (tid == 0) {
        const double tn = nrm[k];
        nrm[k] = nrm[piv];
        nrm[piv] = tn;
        const int ti = perm[k];
        perm[k] = perm[piv];
        perm[piv] = ti;
      }
    }
    __syncthreads();
    double s = 0.0;
    for (int q = k + 1 + tid; q < P; q += NT) {
      const double v = (double)C[(int64_t)q * ldc + k];
      s += v * v;
    }
    s = block_sum(s, red);
    const double alpha = (double)C[(int64_t)k * ldc + k];
    double beta, tau, scal;
    householder(alpha, s, beta, tau, scal);
    for (int q = k + 1 + tid; q < P; q += NT) {
      const T v = (T)((double)C[(int64_t)q * ldc + k] * scal);
      C[(int64_t)q * ldc + k] = v;
      vbuf[q] = (double)v;
    }
    if (tid == 0) {
      vbuf[k] = 1.0;
      d.tauq[k] = (T)tau;
    }
    __syncthreads();
    if (tid == 0) C[(int64_t)k * ldc + k] = (T)beta;
    for (int c = k + 1 + tid; c < m; c += NT) {
      double w = 0.0;
      for (int q = k; q < P; ++q) w += vbuf[q] * (double)C[(int64_t)q * ldc + c];
      const double tw = tau * w;
      double s2 = 0.0;
      for (int q = k; q < P; ++q) {
        const T v = (T)((double)C[(int64_t)q * ldc + c] - tw * vbuf[q]);
        C[(int64_t)q * ldc + c] = v;
        if (q > k) s2 += (double)v * (double)v;
      }
      nrm[c] = s2;
    }
    __syncthreads();
    r = k + 1;
  }
  if (r < P) {
    for (int pos = tid; pos < m; pos += NT) ipos[perm[pos]] = pos;
    __syncthreads();
    // coarse rows W = (Q^T C)[0:r, :] in the original column order
    for (int b = 0; b < nnb; ++b) {
      const int w = off[b + 1] - off[b];
      T* blk = pool + nb[b].blk;
      const int64_t ld = nb[b].ld;
      const int o = off[b];
      if (b < d.nrow) {
        for (int e = tid; e < w * r; e += NT) {
          const int a = e / r, q = e - a * r;
          const int pos = ipos[o + a];
          blk[(int64_t)a * ld + q] = q <= pos ? C[(int64_t)q * ldc + pos] : T(0);
        }
      } else {
        for (int e = tid; e < w * r; e += NT) {
          const int q = e / w, a = e - q * w;
          const int pos = ipos[o + a];
          blk[(int64_t)q * ld + a] = q <= pos ? C[(int64_t)q * ldc + pos] : T(0);
        }
      }
    }
    for (int e = tid; e < P * r; e += NT) {
      const int k = e / P, q = e - k * P;
      d.vq[(int64_t)q + (int64_t)k * P] = q < k ? T(0) : (q == k ? T(1) : C[(int64_t)q * ldc + k]);
    }
    __syncthreads();
    if (tid == 0) rank[d.cluster] = r;
  }
}

// Sparsification for interfaces of at most PMAX unknowns (every interface of
// the 2D workloads): the same steps as k_sparsify, organised for small P and
// wide C.  C is stored column by column with PMAX + 1 rows per column (rows
// P..PMAX zero), in LDS whenever it fits and in the global workspace
// otherwise.  One thread per column: during a step a thread loads its whole
// column into registers from one base address, so the loads overlap instead
// of forming a dependent chain, and needs no predication.  Pivots, column
// norms and the ratio test stay in FP64; ties go to the lowest current
// position (columns are physically swapped).
template <typename T, int PMAX, int NTH>
__global__ void __launch_bounds__(NTH) k_sparsify_small(const SpDesc<T>* __restrict__ descs,
                                                        const SpNbr* __restrict__ nbrs, int lds_c_elems,
                                                        int max_nb) {
  constexpr int NW = NTH / 64;
  constexpr int LDQ = PMAX + 1;
  const SpDesc<T> d = descs[blockIdx.x];
  const double eps = d.eps;
  T* pool = d.pool;
  int* rank = d.rank;
  const int P = d.P, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (P == 0 || *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* bv = reinterpret_cast<double*>(smem);         // NW
  double* sc = bv + NW;                                 // 4 scalars
  int* bi = reinterpret_cast<int*>(sc + 4);             // NW
  T* vb = reinterpret_cast<T*>(smem + align16((size_t)NW * 8 + 32 + (size_t)NW * 4));  // PMAX
  int* off = reinterpret_cast<int*>(vb + PMAX);         // max_nb + 1
  T* Cl = reinterpret_cast<T*>(smem + align16(reinterpret_cast<unsigned char*>(off + max_nb + 1) - smem));
  const int nnb = d.nrow + d.ncol;
  const SpNbr* nb = nbrs + d.nb;
  if (tid == 0) {
    int o = 0;
    for (int b = 0; b < nnb; ++b) {
      off[b] = o;
      o += rank[nb[b].cluster];
    }
    off[nnb] = o;
  }
  __syncthreads();
  const int m = off[nnb];
  T* C = (int64_t)m * LDQ <= (int64_t)lds_c_elems ? Cl : d.C;
  // C[:, o + a]: row a of block (i, p) (row neighbour) or column a of block
  // (p, j) (column neighbour); rows P..PMAX are zero
  for (int b = 0; b < nnb; ++b) {
    const int w = off[b + 1] - off[b];
    const T* blk = pool + nb[b].blk;
    const int64_t ld = nb[b].ld;
    T* Cb = C + (int64_t)off[b] * LDQ;
    const bool rown = b < d.nrow;
    for (int e = tid; e < w * LDQ; e += NTH) {
      const int a = e / LDQ, q = e - a * LDQ;
      T v = T(0);
      if (q < P) v = rown ? blk[(int64_t)a * ld + q] : blk[(int64_t)q * ld + a];
      Cb[e] = v;
    }
  }
  __syncthreads();
  double* nrm = d.nrm;
  int* perm = d.perm;
  int* ipos = d.perm + d.mmax;
  for (int c = tid; c < m; c += NTH) {
    const T* col = C + (int64_t)c * LDQ;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      const double v = (double)col[q];
      s += v * v;
    }
    nrm[c] = s;
    perm[c] = c;
  }
  __syncthreads();
  const int kmax = min(P, m);
  int r = 0;
  double R11 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    double best = -1.0;
    int bidx = m;
    for (int c = k + tid; c < m; c += NTH) {
      const double v = nrm[c];
      if (v > best) {
        best = v;
        bidx = c;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(best, o, 64);
      const int i2 = __shfl_xor(bidx, o, 64);
      if (v2 > best || (v2 == best && i2 < bidx)) {
        best = v2;
        bidx = i2;
      }
    }
    if (lane == 0) {
      bv[wv] = best;
      bi[wv] = bidx;
    }
    __syncthreads();
    if (tid == 0) {
      double b0 = bv[0];
      int i0 = bi[0];
      for (int w = 1; w < NW; ++w)
        if (bv[w] > b0 || (bv[w] == b0 && bi[w] < i0)) {
          b0 = bv[w];
          i0 = bi[w];
        }
      sc[0] = b0;
      sc[2] = (double)i0;
    }
    __syncthreads();
    const int piv = (int)sc[2];
    const double rkk = sqrt(sc[0]);
    __syncthreads();
    if (k == 0) {
      R11 = rkk;
      if (R11 == 0.0) break;
    }
    if (eps > 0.0 && rkk < eps * R11) break;
    if (piv != k) {
      T* ck = C + (int64_t)k * LDQ;
      T* cp = C + (int64_t)piv * LDQ;
      for (int q = tid; q < PMAX; q += NTH) {
        const T a = ck[q];
        ck[q] = cp[q];
        cp[q] = a;
      }
      if (tid == 0) {
        const double tn = nrm[k];
        nrm[k] = nrm[piv];
        nrm[piv] = tn;
        const int ti = perm[k];
        perm[k] = perm[piv];
        perm[piv] = ti;
      }
    }
    __syncthreads();
    if (wv == 0) {
      // Householder of column k (rows k..P-1), one row per lane
      T* ck = C + (int64_t)k * LDQ;
      const double x = lane < P ? (double)ck[lane] : 0.0;
      const double s = wave_sum(lane > k ? x * x : 0.0);
      const double alpha = __shfl(x, k, 64);
      double beta, tau, scal;
      householder(alpha, s, beta, tau, scal);
      if (lane < PMAX) {
        T v;
        if (lane < k) v = T(0);
        else if (lane == k) v = T(1);
        else v = lane < P ? (T)(x * scal) : T(0);
        vb[lane] = v;
        if (lane > k && lane < P) ck[lane] = v;
      }
      if (lane == 0) {
        ck[k] = (T)beta;
        sc[1] = tau;
        d.tauq[k] = (T)tau;
      }
    }
    __syncthreads();
    const T tau = (T)sc[1];
    for (int c = k + 1 + tid; c < m; c += NTH) {
      T* col = C + (int64_t)c * LDQ;
      T a[PMAX];
#pragma unroll
      for (int q = 0; q < PMAX; ++q) a[q] = col[q];
      T w = T(0);
#pragma unroll
      for (int q = 0; q < PMAX; ++q) w += vb[q] * a[q];
      const T tw = tau * w;
      double s2 = 0.0;
#pragma unroll
      for (int q = 0; q < PMAX; ++q) {
        a[q] -= tw * vb[q];
        const double aq = (double)a[q];
        s2 += q > k ? aq * aq : 0.0;
      }
#pragma unroll
      for (int q = 0; q < PMAX; ++q) col[q] = a[q];
      nrm[c] = s2;
    }
    __syncthreads();
    r = k + 1;
  }
  if (r < P) {
    for (int pos = tid; pos < m; pos += NTH) ipos[perm[pos]] = pos;
    __syncthreads();
    for (int b = 0; b < nnb; ++b) {
      const int w = off[b + 1] - off[b];
      T* blk = pool + nb[b].blk;
      const int64_t ld = nb[b].ld;
      const int o = off[b];
      if (b < d.nrow) {
        for (int e = tid; e < w * r; e += NTH) {
          const int a = e / r, q = e - a * r;
          const int pos = ipos[o + a];
          blk[(int64_t)a * ld + q] = q <= pos ? C[(int64_t)pos * LDQ + q] : T(0);
        }
      } else {
        for (int e = tid; e < w * r; e += NTH) {
          const int q = e / w, a = e - q * w;
          const int pos = ipos[o + a];
          blk[(int64_t)q * ld + a] = q <= pos ? C[(int64_t)pos * LDQ + q] : T(0);
        }
      }
    }
    for (int e = tid; e < P * r; e += NTH) {
      const int k = e / P, q = e - k * P;
      d.vq[(int64_t)q + (int64_t)k * P] = q < k ? T(0) : (q == k ? T(1) : C[(int64_t)k * LDQ + q]);
    }
    __syncthreads();
    if (tid == 0) rank[d.cluster] = r;
  }
}

// Register-resident partial CPQR of C = [A_np^T | A_pn] (Sections 2.5, 2.6;
// rank rule of Section 4).  Thread tid owns columns tid + SP_NT j: j < CPT in
// registers and, if LC, one more column in LDS (element q at
// q * SP_NT + tid, conflict-free), for the whole factorization (P <= PMAX
// rows each), and, if GC, one more in global memory (the descriptor's
// workspace C, element q at q * SP_NT + tid).  Columns are never moved: each carries its current position,
// and the swap of the pivot with the column at position k only exchanges
// positions, so the pivot choice (largest FP64 norm, ties to the lowest
// current position) is the same as with physical swaps.  Per step: local and
// wavefront argmax, the winning lane of each wavefront stages its column in
// LDS, one barrier, the workgroup winner is picked, wavefront 0 forms the
// Householder vector (dlarfg convention) in LDS, a second barrier, then every
// live column is updated and its tail norm recomputed in FP64.  The pivot
// column keeps R above the diagonal and becomes beta at row k.  After r steps
// rows 0..r-1 of every column are W = Q^T C (zero below the diagonal of pivot
// columns) and go back to the blocks.
constexpr int SP_NT = 512;

template <typename T, int PMAX, int CPT, int LC, int GC>
__global__ void __launch_bounds__(SP_NT) k_cpqr_reg(const SpDesc<T>* __restrict__ descs,
                                                    const SpNbr* __restrict__ nbrs, int max_nb) {
  constexpr int NW = SP_NT / 64;
  constexpr int NCL = CPT + LC;     // columns in registers and LDS
  constexpr int NC = NCL + GC;      // and in global memory
  constexpr int VN = Vec16<T>::N;
  const SpDesc<T> d = descs[blockIdx.x];
  const double eps = d.eps;
  T* pool = d.pool;
  int* rank = d.rank;
  const int P = d.P, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (P == 0 || *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* slot = reinterpret_cast<T*>(smem);                       // 2 x NW x PMAX
  T* vbuf = slot + 2 * NW * PMAX;                             // PMAX
  T* lcol = vbuf + PMAX;                                      // LC ? PMAX x SP_NT : 0
  double* cb = reinterpret_cast<double*>(lcol + LC * PMAX * SP_NT);  // 2 x NW candidate norms
  double* hs = cb + 2 * NW;                                   // tau, beta
  int* cpz = reinterpret_cast<int*>(hs + 2);                  // 2 x NW candidate positions
  int* off = cpz + 2 * NW;                                    // max_nb + 1
  const int nnb = d.nrow + d.ncol;
  const SpNbr* nb = nbrs + d.nb;
  if (tid == 0) {
    int o = 0;
    for (int b = 0; b < nnb; ++b) {
      off[b] = o;
      o += rank[nb[b].cluster];
    }
    off[nnb] = o;
  }
  __syncthreads();
  const int m = off[nnb];
  // column c of C: row ai of block (i, p) for a row neighbour, column ai of
  // block (p, j) for a column neighbour
  auto col_src = [&](int c, int64_t& str) -> T* {
    int b = 0;
    while (off[b + 1] <= c) ++b;
    const int ai = c - off[b];
    T* blk = pool + nb[b].blk;
    const int64_t ld = nb[b].ld;
    str = b < d.nrow ? 1 : ld;
    return b < d.nrow ? blk + (int64_t)ai * ld : blk + ai;
  };
  T a[CPT][PMAX];
  double nr[NC];
  int pos[NC], kel[NC];
  T* lc = lcol + tid;  // the LDS column, stride SP_NT
  T* gcp = GC ? d.C + tid : nullptr;  // the global column, stride SP_NT (touched only when it exists)
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const int c = tid + SP_NT * j;
    pos[j] = c;
    kel[j] = -1;
    int64_t str = 0;
    const T* src = c < m ? col_src(c, str) : nullptr;
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < PMAX; ++q) {
      const T x = (src && q < P) ? src[q * str] : T(0);
      if (j < CPT) a[j < CPT ? j : 0][q] = x;
      else if (j < NCL) lc[q * SP_NT] = x;
      else if (c < m) gcp[q * SP_NT] = x;
      s2 += (double)x * (double)x;
    }
    nr[j] = c < m ? s2 : -1.0;
  }
  const int kmax = min(P, m);
  int r = 0;
  double R11 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    const int buf = k & 1;
    double best = -1.0;
    int bp = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (kel[j] < 0 && nr[j] >= 0.0 && (nr[j] > best || (nr[j] == best && pos[j] < bp))) {
        best = nr[j];
        bp = pos[j];
      }
    double wb = best;
    int wp = bp;
    {
      auto merge = [&](double ob, int op) {
        if (ob > wb || (ob == wb && op < wp)) {
          wb = ob;
          wp = op;
        }
      };
      merge(xshfl<32>(wb), xshfl<32>(wp));
      merge(xshfl<16>(wb), xshfl<16>(wp));
      merge(xshfl<8>(wb), xshfl<8>(wp));
      merge(xshfl<4>(wb), xshfl<4>(wp));
      merge(xshfl<2>(wb), xshfl<2>(wp));
      merge(xshfl<1>(wb), xshfl<1>(wp));
    }
    if (wp != 0x7fffffff && bp == wp) {
      T* sl = slot + (buf * NW + wv) * PMAX;
#pragma unroll
      for (int j = 0; j < NC; ++j)
        if (kel[j] < 0 && pos[j] == wp) {
          if (j < CPT) {
            lds_store_row<T, PMAX>(sl, a[j < CPT ? j : 0]);
          } else if (j < NCL) {
            for (int q = 0; q < PMAX; ++q) sl[q] = lc[q * SP_NT];
          } else {
            for (int q = 0; q < PMAX; ++q) sl[q] = gcp[q * SP_NT];
          }
        }
    }
    if (lane == 0) {
      cb[buf * NW + wv] = wb;
      cpz[buf * NW + wv] = wp;
    }
    __syncthreads();
    int ws = 0;
    double gb = cb[buf * NW];
    int gp = cpz[buf * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const double ob = cb[buf * NW + w];
      const int op = cpz[buf * NW + w];
      if (ob > gb || (ob == gb && op < gp)) {
        gb = ob;
        gp = op;
        ws = w;
      }
    }
    const double rkk = sqrt(gb);
    if (k == 0) {
      R11 = rkk;
      if (R11 == 0.0) break;
    }
    if (eps > 0.0 && rkk < eps * R11) break;
    if (wv == 0) {
      const double x = lane < P ? (double)slot[(buf * NW + ws) * PMAX + lane] : 0.0;
      const double s = wave_sum(lane > k ? x * x : 0.0);
      const double alpha = __shfl(x, k, 64);
      double beta, tau, scal;
      householder(alpha, s, beta, tau, scal);
      const double v = lane < k ? 0.0 : (lane == k ? 1.0 : x * scal);
      if (lane < PMAX) vbuf[lane] = (T)v;
      if (lane < P) d.vq[(int64_t)lane + (int64_t)k * P] = (T)v;
      if (lane == 0) {
        hs[0] = tau;
        hs[1] = beta;
        d.tauq[k] = (T)tau;
      }
    }
    __syncthreads();
    const T tau = (T)hs[0], beta = (T)hs[1];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (kel[j] >= 0 || nr[j] < 0.0) continue;
      if (pos[j] == gp) {
        // the pivot: beta at row k, reflector storage below (not part of W)
        kel[j] = k;
        pos[j] = k;
        if (j < CPT) {
#pragma unroll
          for (int q = 0; q < PMAX; ++q) a[j < CPT ? j : 0][q] = q == k ? beta : a[j < CPT ? j : 0][q];
        } else if (j < NCL) {
          lc[k * SP_NT] = beta;
        } else {
          gcp[k * SP_NT] = beta;
        }
        continue;
      }
      if (pos[j] == k) pos[j] = gp;
      T w = T(0);
      double s2 = 0.0;
      if (j < CPT) {
        T(&aj)[PMAX] = a[j < CPT ? j : 0];
#pragma unroll
        for (int q0 = 0; q0 < PMAX; q0 += VN) {
          if (q0 + VN - 1 < k) continue;  // v is zero there (uniform)
          T vv[VN];
          Vec16<T>::put(*reinterpret_cast<const typename Vec16<T>::type*>(vbuf + q0), vv);
#pragma unroll
          for (int e = 0; e < VN; ++e) w += vv[e] * aj[q0 + e];
        }
        const T tw = tau * w;
#pragma unroll
        for (int q0 = 0; q0 < PMAX; q0 += VN) {
          if (q0 + VN - 1 < k) continue;
          T vv[VN];
          Vec16<T>::put(*reinterpret_cast<const typename Vec16<T>::type*>(vbuf + q0), vv);
#pragma unroll
          for (int e = 0; e < VN; ++e) {
            aj[q0 + e] -= tw * vv[e];
            const double x = (double)aj[q0 + e];
            s2 += q0 + e > k ? x * x : 0.0;
          }
        }
      } else {
        T* cp = j < NCL ? lc : gcp;
        for (int q = k; q < PMAX; ++q) w += vbuf[q] * cp[q * SP_NT];
        const T tw = tau * w;
        for (int q = k; q < PMAX; ++q) {
          const T x = cp[q * SP_NT] - tw * vbuf[q];
          cp[q * SP_NT] = x;
          if (q > k) s2 += (double)x * (double)x;
        }
      }
      nr[j] = s2;
    }
    r = k + 1;
  }
  if (r < P) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = tid + SP_NT * j;
      if (c >= m) continue;
      int64_t str = 0;
      T* dst = col_src(c, str);
#pragma unroll
      for (int q = 0; q < PMAX; ++q)
        if (q < r) {
          const T x = j < CPT ? a[j < CPT ? j : 0][q] : (j < NCL ? lc[q * SP_NT] : gcp[q * SP_NT]);
          dst[q * str] = (kel[j] >= 0 && q > kel[j]) ? T(0) : x;
        }
    }
    if (tid == 0) rank[d.cluster] = r;
  }
}

// Cooperative partial CPQR (same method and pivot rule as k_cpqr_reg) for
// interfaces whose columns do not fit one workgroup.  Every workgroup is one
// wavefront owning columns (g cpt + j) 64 + lane of its interface; C is
// row-major in global memory (coalesced rows, mostly L2-resident).  Per pivot
// step: each workgroup publishes its best live column (FP64 norm, position,
// values) in a double-buffered slot, one grid-wide barrier, then every
// workgroup of the interface picks the same winner, forms the Householder
// vector (dlarfg convention) in LDS and updates its own columns.  Interfaces
// that stopped keep taking part in the barriers; the loop ends for the whole
// grid once every interface has reported done (flags double-buffered by step
// parity, so all workgroups read the same flags after a barrier).
// Barrier of the nblk workgroups that factor one interface together (all
// co-resident: the launch is cooperative).  cnt counts arrivals, gen is the
// generation the waiters watch; the last to arrive resets cnt and advances
// gen.  Each interface has its own pair, so interfaces of one launch never
// wait for each other.
__device__ __forceinline__ void team_sync(int* cnt, int* gen, int nblk) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(cnt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == nblk - 1) {
      __hip_atomic_store(cnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      // relaxed polling (no cache invalidation per poll), one acquire after
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) __builtin_amdgcn_s_sleep(1);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

template <typename T, int CPT, bool LC>
__global__ void __launch_bounds__(64) k_cpqr_coop(const SpDesc<T>* __restrict__ descs, const SpNbr* __restrict__ nbrs,
                                                 const CoopItem* __restrict__ items, int nitems, int total_blocks,
                                                 int max_p, int max_nb, double* ckey, int* cpos, T* ccol, int* done,
                                                 int kmax_all) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* vbuf = reinterpret_cast<T*>(smem);                      // max_p
  T* cl = vbuf + ((max_p + 3) & ~3);                          // LC: P x 64 CPT, this workgroup's columns
  int* off = reinterpret_cast<int*>(cl + (LC ? (size_t)max_p * 64 * CPT : 0));  // max_nb + 1
  const int b = blockIdx.x, lane = threadIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b) lo = mid;
    else hi = mid - 1;
  }
  const int it = lo;
  const CoopItem ci = items[it];
  const SpDesc<T> d = descs[it];
  const int g = b - ci.first;
  const int P = d.P;
  // columns live in LDS (LC: local index j 64 + lane, leading dimension
  // 64 CPT) or in the row-major global workspace (global index)
  const int64_t ldm = LC ? 64 * CPT : d.mmax;
  T* C = LC ? cl : d.C;
  auto cidx = [&](int j) { return LC ? j * 64 + lane : (g * CPT + j) * 64 + lane; };
  const int nnb = d.nrow + d.ncol;
  const SpNbr* nb = nbrs + d.nb;
  bool fin = !(P > 0 && *d.flag == 0);  // not scaled: rank stays P, nothing to do
  if (lane == 0) {
    int o = 0;
    for (int q = 0; q < nnb; ++q) {
      off[q] = o;
      o += d.rank[nb[q].cluster];
    }
    off[nnb] = o;
  }
  __syncthreads();
  const int m = off[nnb];
  auto col_src = [&](int c, int64_t& str) -> T* {
    int q = 0;
    while (off[q + 1] <= c) ++q;
    const int ai = c - off[q];
    T* blk = d.pool + nb[q].blk;
    const int64_t ld = nb[q].ld;
    str = q < d.nrow ? 1 : ld;
    return q < d.nrow ? blk + (int64_t)ai * ld : blk + ai;
  };
  double nr[CPT];
  int pos[CPT], kel[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = (g * CPT + j) * 64 + lane;
    pos[j] = c;
    kel[j] = -1;
    nr[j] = -1.0;
    if (!fin && c < m) {
      int64_t str = 0;
      const T* src = col_src(c, str);
      double s2 = 0.0;
      const int ci = cidx(j);
      for (int q0 = 0; q0 < P; q0 += 16) {
        T x[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = q0 + e < P ? src[(int64_t)(q0 + e) * str] : T(0);
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (q0 + e < P) {
            C[(int64_t)(q0 + e) * ldm + ci] = x[e];
            s2 += (double)x[e] * (double)x[e];
          }
      }
      nr[j] = s2;
    }
  }
  // an interface that is not scaled keeps its size: its whole team leaves
  // at once (fin is the same on every workgroup of the team)
  const int kmax = min(P, m);
  int r = 0;
  double R11 = 0.0;
  int* bar = done + 2 * it;  // this interface's barrier: arrivals, generation
  for (int k = 0; !fin && k <= kmax_all; ++k) {
    const int buf = k & 1;
    // this workgroup's best live column: (norm desc, position asc)
    double wb = -1.0;
    int wp = 0x7fffffff, wc = -1;
#pragma unroll
      for (int j = 0; j < CPT; ++j)
        if (kel[j] < 0 && nr[j] >= 0.0 && (nr[j] > wb || (nr[j] == wb && pos[j] < wp))) {
          wb = nr[j];
          wp = pos[j];
          wc = cidx(j);
        }
    {
      auto merge = [&](double ob, int op, int oc) {
        if (ob > wb || (ob == wb && op < wp)) {
          wb = ob;
          wp = op;
          wc = oc;
        }
      };
      merge(xshfl<32>(wb), xshfl<32>(wp), xshfl<32>(wc));
      merge(xshfl<16>(wb), xshfl<16>(wp), xshfl<16>(wc));
      merge(xshfl<8>(wb), xshfl<8>(wp), xshfl<8>(wc));
      merge(xshfl<4>(wb), xshfl<4>(wp), xshfl<4>(wc));
      merge(xshfl<2>(wb), xshfl<2>(wp), xshfl<2>(wc));
      merge(xshfl<1>(wb), xshfl<1>(wp), xshfl<1>(wc));
    }
    T* cc = ccol + ((int64_t)buf * total_blocks + b) * max_p;
    if (wc >= 0)
      for (int q = lane; q < P; q += 64) cc[q] = C[(int64_t)q * ldm + wc];
    if (lane == 0) {
      ckey[buf * total_blocks + b] = wb;
      cpos[buf * total_blocks + b] = wp;
    }
    team_sync(bar, bar + 1, ci.nblk);
    {
      // the interface's winner among its workgroups
      double gb = -1.0;
      int gp = 0x7fffffff, gw = -1;
      for (int w = lane; w < ci.nblk; w += 64) {
        const double ob = ckey[buf * total_blocks + ci.first + w];
        const int op = cpos[buf * total_blocks + ci.first + w];
        if (ob > gb || (ob == gb && op < gp)) {
          gb = ob;
          gp = op;
          gw = w;
        }
      }
      {
        auto merge = [&](double ob, int op, int ow) {
          if (ob > gb || (ob == gb && op < gp)) {
            gb = ob;
            gp = op;
            gw = ow;
          }
        };
        merge(xshfl<32>(gb), xshfl<32>(gp), xshfl<32>(gw));
        merge(xshfl<16>(gb), xshfl<16>(gp), xshfl<16>(gw));
        merge(xshfl<8>(gb), xshfl<8>(gp), xshfl<8>(gw));
        merge(xshfl<4>(gb), xshfl<4>(gp), xshfl<4>(gw));
        merge(xshfl<2>(gb), xshfl<2>(gp), xshfl<2>(gw));
        merge(xshfl<1>(gb), xshfl<1>(gp), xshfl<1>(gw));
      }
      const double rkk = sqrt(max(gb, 0.0));
      if (k == 0) R11 = rkk;
      const bool stop = k >= kmax || gw < 0 || R11 == 0.0 || (d.eps > 0.0 && rkk < d.eps * R11);
      if (stop) {
        fin = true;
      } else {
        const T* xw = ccol + ((int64_t)buf * total_blocks + ci.first + gw) * max_p;
        double s = 0.0, alpha = 0.0;
        for (int q = lane; q < P; q += 64) {
          const double x = (double)xw[q];
          if (q > k) s += x * x;
          if (q == k) alpha = x;
        }
        s = wave_sum(s);
        alpha = wave_sum(alpha);
        double beta, tau, scal;
        householder(alpha, s, beta, tau, scal);
        for (int q = lane; q < P; q += 64) {
          const double v = q < k ? 0.0 : (q == k ? 1.0 : (double)xw[q] * scal);
          vbuf[q] = (T)v;
          if (g == 0) d.vq[(int64_t)q + (int64_t)k * P] = (T)v;
        }
        if (g == 0 && lane == 0) d.tauq[k] = (T)tau;
        __syncthreads();
        const T tt = (T)tau, bt = (T)beta;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
          if (kel[j] >= 0 || nr[j] < 0.0) continue;
          const int c = cidx(j);
          if (pos[j] == gp) {
            kel[j] = k;
            pos[j] = k;
            C[(int64_t)k * ldm + c] = bt;
            continue;
          }
          if (pos[j] == k) pos[j] = gp;
          // rows k..P-1 in chunks of 16 independent loads
          constexpr int CH = 16;
          T w = T(0);
          for (int q0 = k; q0 < P; q0 += CH) {
            T x[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) x[e] = q0 + e < P ? C[(int64_t)(q0 + e) * ldm + c] : T(0);
#pragma unroll
            for (int e = 0; e < CH; ++e) w += (q0 + e < P ? vbuf[q0 + e] : T(0)) * x[e];
          }
          const T tw = tt * w;
          double s2 = 0.0;
          for (int q0 = k; q0 < P; q0 += CH) {
            T x[CH];
#pragma unroll
            for (int e = 0; e < CH; ++e) x[e] = q0 + e < P ? C[(int64_t)(q0 + e) * ldm + c] : T(0);
#pragma unroll
            for (int e = 0; e < CH; ++e)
              if (q0 + e < P) {
                const T y = x[e] - tw * vbuf[q0 + e];
                C[(int64_t)(q0 + e) * ldm + c] = y;
                if (q0 + e > k) s2 += (double)y * (double)y;
              }
          }
          nr[j] = s2;
        }
        r = k + 1;
        __syncthreads();
      }
    }
  }
  if (P > 0 && *d.flag == 0 && r < P) {
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const int c = (g * CPT + j) * 64 + lane;
      if (c >= m) continue;
      int64_t str = 0;
      T* dst = col_src(c, str);
      const int ci = cidx(j);
      for (int q = 0; q < r; ++q) dst[q * str] = (kel[j] >= 0 && q > kel[j]) ? T(0) : C[(int64_t)q * ldm + ci];
    }
    if (g == 0 && lane == 0) d.rank[d.cluster] = r;
  }
}

// ---------------------------------------------------------------- apply
// Rows of a work vector are owned by lane (row % 64) for the whole kernel, so
// a wavefront needs no barrier between reflectors.
template <typename T, bool UNIT_STORED>
__device__ void wave_reflectors(const T* __restrict__ V, int64_t ldv, const T* __restrict__ tau, int first,
                                int last, int step, int m, double* xs, int nc, int ldx) {
  const int lane = threadIdx.x & 63;
  for (int t = first; t != last; t += step) {
    const double tt = (double)tau[t];
    if (tt == 0.0) continue;
    const T* v = V + (int64_t)t * ldv;
    double acc[RBMAX];
#pragma unroll
    for (int c = 0; c < RBMAX; ++c) acc[c] = 0.0;
    for (int r = (t & ~63) + lane; r < m; r += 64) {
      if (r < t) continue;
      const double vr = (r == t && !UNIT_STORED) ? 1.0 : (double)v[r];
#pragma unroll
      for (int c = 0; c < RBMAX; ++c)
        if (c < nc) acc[c] += vr * xs[r + c * ldx];
    }
#pragma unroll
    for (int c = 0; c < RBMAX; ++c)
      if (c < nc) acc[c] = tt * wave_sum(acc[c]);
    for (int r = (t & ~63) + lane; r < m; r += 64) {
      if (r < t) continue;
      const double vr = (r == t && !UNIT_STORED) ? 1.0 : (double)v[r];
#pragma unroll
      for (int c = 0; c < RBMAX; ++c)
        if (c < nc) xs[r + c * ldx] -= acc[c] * vr;
    }
  }
}

// x <- R^{-1} x, R upper triangular n x n column-major (ld), x in LDS.
template <typename T>
__device__ void wave_backsolve(const T* __restrict__ R, int64_t ld, int n, double* xs, int nc, int ldx) {
  const int lane = threadIdx.x & 63;
  for (int c = n - 1; c >= 0; --c) {
    const double d = (double)R[c + (int64_t)c * ld];
    if (lane == (c & 63))
      for (int q = 0; q < nc; ++q) xs[c + q * ldx] /= d;
    __syncthreads();
    const T* Rc = R + (int64_t)c * ld;
    for (int r = lane; r < c; r += 64) {
      const double rv = (double)Rc[r];
      for (int q = 0; q < nc; ++q) xs[r + q * ldx] -= rv * xs[c + q * ldx];
    }
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(64) k_ap_front_fwd(const ApFront<T>* __restrict__ ds, double* x,
                                                    int64_t ldx, int nrhs, int rb) {
  const ApFront<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.n == 0 || nc <= 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* xs = reinterpret_cast<double*>(smem);
  const int m = d.m, lane = threadIdx.x;
  for (int c = 0; c < nc; ++c)
    for (int r = lane; r < m; r += 64) xs[r + c * m] = x[d.rows[r] + (int64_t)(c0 + c) * ldx];
  wave_reflectors<T, false>(d.vr, m, d.tau, 0, d.n, 1, m, xs, nc, m);
  for (int c = 0; c < nc; ++c)
    for (int r = lane; r < m; r += 64) x[d.rows[r] + (int64_t)(c0 + c) * ldx] = xs[r + c * m];
}

template <typename T>
__global__ void __launch_bounds__(64) k_ap_front_bwd(const ApFront<T>* __restrict__ ds, double* x,
                                                    int64_t ldx, int nrhs, int rb) {
  const ApFront<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.n == 0 || nc <= 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = d.n, k = d.k, lane = threadIdx.x;
  double* ys = reinterpret_cast<double*>(smem);  // n x nc
  double* xc = ys + (size_t)n * rb;              // k x nc
  for (int c = 0; c < nc; ++c) {
    for (int r = lane; r < n; r += 64) ys[r + c * n] = x[d.rows[r] + (int64_t)(c0 + c) * ldx];
    for (int r = lane; r < k; r += 64) xc[r + c * k] = x[d.cols[r] + (int64_t)(c0 + c) * ldx];
  }
  __syncthreads();
  // y_s -= R_sj x_j
  for (int j = 0; j < k; ++j) {
    const T* col = d.rsj + (int64_t)j * n;
    for (int r = lane; r < n; r += 64) {
      const double rv = (double)col[r];
      for (int c = 0; c < nc; ++c) ys[r + c * n] -= rv * xc[j + c * k];
    }
  }
  __syncthreads();
  wave_backsolve<T>(d.vr, d.m, n, ys, nc, n);
  for (int c = 0; c < nc; ++c)
    for (int r = lane; r < n; r += 64) x[d.rows[r] + (int64_t)(c0 + c) * ldx] = ys[r + c * n];
}

template <typename T>
__global__ void __launch_bounds__(64) k_ap_iface_fwd(const ApIface<T>* __restrict__ ds, double* x,
                                                    int64_t ldx, int nrhs, int rb) {
  const ApIface<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.P == 0 || nc <= 0 || *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* xs = reinterpret_cast<double*>(smem);
  const int P = d.P, lane = threadIdx.x, r = *d.rank;
  for (int c = 0; c < nc; ++c)
    for (int q = lane; q < P; q += 64) xs[q + c * P] = x[d.slots[q] + (int64_t)(c0 + c) * ldx];
  wave_reflectors<T, false>(d.vru, P, d.tauu, 0, P, 1, P, xs, nc, P);
  if (r < P) wave_reflectors<T, true>(d.vq, P, d.tauq, 0, r, 1, P, xs, nc, P);
  for (int c = 0; c < nc; ++c)
    for (int q = lane; q < P; q += 64) x[d.slots[q] + (int64_t)(c0 + c) * ldx] = xs[q + c * P];
}

template <typename T>
__global__ void __launch_bounds__(64) k_ap_iface_bwd(const ApIface<T>* __restrict__ ds, double* x,
                                                    int64_t ldx, int nrhs, int rb) {
  const ApIface<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.P == 0 || nc <= 0 || *d.flag != 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  double* xs = reinterpret_cast<double*>(smem);
  const int P = d.P, lane = threadIdx.x, r = *d.rank;
  for (int c = 0; c < nc; ++c)
    for (int q = lane; q < P; q += 64) xs[q + c * P] = x[d.slots[q] + (int64_t)(c0 + c) * ldx];
  if (r < P) wave_reflectors<T, true>(d.vq, P, d.tauq, r - 1, -1, -1, P, xs, nc, P);
  __syncthreads();
  wave_backsolve<T>(d.vru, P, P, xs, nc, P);
  for (int c = 0; c < nc; ++c)
    for (int q = lane; q < P; q += 64) x[d.slots[q] + (int64_t)(c0 + c) * ldx] = xs[q + c * P];
}

// Forward sweep of one colour of fronts, panel by panel with the compact-WY
// factors stored by the QR: x[rows] <- (I - V_p T_p V_p^T)^T x[rows] for the
// panels p = 0, 1, ...  Four wavefronts per front; a panel costs one pass of
// independent loads for V_p^T x and one (cached) pass for the update, instead
// of two dependent passes per reflector.
template <typename T, int JB>
__global__ void __launch_bounds__(256) k_ap_front_fwd_wy(const ApFront<T>* __restrict__ ds, double* x, int64_t ldx,
                                                        int nrhs, int rb) {
  const ApFront<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.n == 0 || nc <= 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int m = d.m, n = d.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* xs = reinterpret_cast<double*>(smem);  // m x nc
  double* red = xs + (size_t)m * rb;             // 4 x JB
  double* wb = red + 4 * JB;                     // JB
  double* ub = wb + JB;                          // JB
  for (int c = 0; c < nc; ++c)
    for (int r = tid; r < m; r += 256) xs[r + c * m] = x[d.rows[r] + (int64_t)(c0 + c) * ldx];
  __syncthreads();
  for (int p0 = 0; p0 < n; p0 += JB) {
    const int jb = min(JB, n - p0);
    const T* Vp = d.vr + (int64_t)p0 * m;
    const T* Tp = d.tpan + (int64_t)(p0 / JB) * JB * JB;
    for (int c = 0; c < nc; ++c) {
      double acc[JB];
#pragma unroll
      for (int t = 0; t < JB; ++t) acc[t] = 0.0;
      for (int r = p0 + tid; r < m; r += 256) {
        const double xr = xs[r + c * m];
        const int rr = r - p0;
#pragma unroll
        for (int t = 0; t < JB; ++t) {
          const double v = (t >= jb || rr < t) ? 0.0 : (rr == t ? 1.0 : (double)Vp[r + (int64_t)t * m]);
          acc[t] += v * xr;
        }
      }
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const double sv = wave_sum(acc[t]);
        if (lane == 0) red[wv * JB + t] = sv;
      }
      __syncthreads();
      if (tid < JB) wb[tid] = red[tid] + red[JB + tid] + red[2 * JB + tid] + red[3 * JB + tid];
      __syncthreads();
      if (tid < JB) {
        double u = 0.0;
        for (int q = 0; q <= tid; ++q) u += (double)Tp[q + tid * JB] * wb[q];
        ub[tid] = u;
      }
      __syncthreads();
      for (int r = p0 + tid; r < m; r += 256) {
        const int rr = r - p0;
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < JB; ++t) {
          const double v = (t >= jb || rr < t) ? 0.0 : (rr == t ? 1.0 : (double)Vp[r + (int64_t)t * m]);
          s += v * ub[t];
        }
        xs[r + c * m] -= s;
      }
      __syncthreads();
    }
  }
  for (int c = 0; c < nc; ++c)
    for (int r = tid; r < m; r += 256) x[d.rows[r] + (int64_t)(c0 + c) * ldx] = xs[r + c * m];
}

// Backward sweep of the fronts of one level: x_s <- R_ss^{-1} (x_s - R_sj x_j).
// The R_sj product: the rows of the front spread over the workgroup's
// threads and, when the front has fewer than 256 rows, its columns j over
// G = 256 / rows' groups (shorter load chains), partial sums combined in LDS;
// the triangular solve runs in 64-row blocks from the bottom, each diagonal
// block by one wavefront with shuffles, the rows above it updated by all
// threads.
constexpr int kBwdTile = 128;   // largest number of rows of the LDS tile of R_ss in the backward apply
constexpr int kBwdChunk = 1024; // largest number of ancestor unknowns x_j staged in LDS at a time

template <typename T>
__global__ void __launch_bounds__(256) k_ap_front_bwd_reg(const ApFront<T>* __restrict__ ds, double* x,
                                                         int64_t ldx, int nrhs, int rb, int chunk, int tile_rows) {
  const ApFront<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * rb, nc = min(rb, nrhs - c0);
  if (d.n == 0 || nc <= 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = d.n, k = d.k, m = d.m, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* ys = reinterpret_cast<double*>(smem);  // n x nc
  double* xc = ys + (size_t)n * rb;              // chunk x nc: x_j, chunk by chunk
  double* part = xc + (size_t)chunk * rb;        // 256 partial sums
  for (int c = 0; c < nc; ++c)
    for (int r = tid; r < n; r += 256) ys[r + c * n] = x[d.rows[r] + (int64_t)(c0 + c) * ldx];
  {
    // rows per pass RP (64, 128 or 256: a divisor of the workgroup size, so
    // every thread has exactly one row and group), column groups G = 256 / RP
    const int RP = n <= 64 ? 64 : (n <= 128 ? 128 : 256);
    const int G = 256 / RP, r0 = tid % RP, g = tid / RP;
    for (int j0 = 0; j0 < k; j0 += chunk) {
      const int kc = min(chunk, k - j0);
      for (int c = 0; c < nc; ++c)
        for (int r = tid; r < kc; r += 256) xc[r + c * chunk] = x[d.cols[j0 + r] + (int64_t)(c0 + c) * ldx];
      __syncthreads();
      for (int c = 0; c < nc; ++c)
        for (int rbase = 0; rbase < n; rbase += RP) {
          const int r = rbase + r0;
          double acc = 0.0;
          if (r < n) {
            const T* rc = d.rsj + r + (int64_t)j0 * n;
#pragma unroll 8
            for (int j = g; j < kc; j += G) acc += (double)rc[(int64_t)j * n] * xc[j + c * chunk];
          }
          if (G == 1) {
            if (r < n) ys[r + c * n] -= acc;
          } else {
            part[g * RP + r0] = acc;
            __syncthreads();
            if (g == 0 && r < n) {
              double t = 0.0;
              for (int h = 0; h < G; ++h) t += part[h * RP + r0];
              ys[r + c * n] -= t;
            }
            __syncthreads();
          }
        }
      __syncthreads();
    }
  }
  __syncthreads();
  // R_ss (column-major in vr, leading dimension m) is staged through an LDS
  // tile of tile_rows (64 or 128) rows x 64 columns: every load of a block is
  // issued at once by the whole workgroup instead of one dependent chain per
  // thread
  const T* R = d.vr;
  T* Rt = reinterpret_cast<T*>(part + 256);  // tile_rows x 65
  for (int b0 = ((n - 1) / 64) * 64; b0 >= 0; b0 -= 64) {
    const int b1 = min(n, b0 + 64), bw = b1 - b0;
    for (int q = tid; q < 64 * 64; q += 256) {
      const int r = q & 63, cc = q >> 6;
      Rt[r * 65 + cc] = (r < bw && cc < bw) ? R[(b0 + r) + (int64_t)(b0 + cc) * m] : T(0);
    }
    __syncthreads();
    if (wv == 0) {
      const int row = b0 + lane;
      for (int c = 0; c < nc; ++c) {
        double yl = row < b1 ? ys[row + c * n] : 0.0;
        for (int lc = bw - 1; lc >= 0; --lc) {
          if (lane == lc) yl = yl / (double)Rt[lc * 65 + lc];
          const double yc = __shfl(yl, lc, 64);
          if (lane < lc) yl -= (double)Rt[lane * 65 + lc] * yc;
        }
        if (row < b1) ys[row + c * n] = yl;
      }
    }
    __syncthreads();
    for (int rs = 0; rs < b0; rs += tile_rows) {
      const int nr = min(tile_rows, b0 - rs);
      for (int q = tid; q < nr * bw; q += 256) {
        const int cc = q / nr, r = q - cc * nr;
        Rt[r * 65 + cc] = R[(rs + r) + (int64_t)(b0 + cc) * m];
      }
      __syncthreads();
      for (int c = 0; c < nc; ++c)
        for (int r = tid; r < nr; r += 256) {
          double sacc = 0.0;
          for (int cc = 0; cc < bw; ++cc) sacc += (double)Rt[r * 65 + cc] * ys[b0 + cc + c * n];
          ys[rs + r + c * n] -= sacc;
        }
      __syncthreads();
    }
  }
  for (int c = 0; c < nc; ++c)
    for (int r = tid; r < n; r += 256) x[d.rows[r] + (int64_t)(c0 + c) * ldx] = ys[r + c * n];
}

// Forward apply of a front, x[rows] <- H_s^T x[rows], with the rows held in
// registers: thread tid owns front rows tid + 256 q, q < Q (m <= 256 Q), and
// NR right-hand sides.  Per JB-reflector panel: w = V^T x is reduced over the
// workgroup in one reduce-scatter and one barrier, lane t of each wavefront
// forms u_t = (T^T w)_t from column t of the compact-WY factor, the u values
// are broadcast with readlane, and x <- x - V u.  The next panel's V is
// loaded while the current one is applied.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <typename T, int JB, int Q, int NR>
__global__ void __launch_bounds__(256) k_ap_front_fwd_reg(const ApFront<T>* __restrict__ ds, double* x, int64_t ldx,
                                                         int nrhs) {
  constexpr int K = JB * NR;  // reduced values per panel, at most 64
  constexpr int SH = 6 - ilog2c(K);
  static_assert(K <= 64, "panel values exceed one wavefront");
  __shared__ __align__(16) double red[2][4][K];
  const ApFront<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int c0 = blockIdx.y * NR;
  if (d.n == 0 || c0 >= nrhs) return;
  const int nc = min(NR, nrhs - c0);
  const int m = d.m, n = d.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double xr[Q][NR];
  int sl[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = tid + 256 * q;
    sl[q] = r < m ? d.rows[r] : 0;
#pragma unroll
    for (int c = 0; c < NR; ++c) xr[q][c] = (r < m && c < nc) ? x[sl[q] + (int64_t)(c0 + c) * ldx] : 0.0;
  }
  T vc[Q][JB];
  auto load_v = [&](int p0, T (&v)[Q][JB]) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int r = tid + 256 * q, rr = r - p0;
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const bool col = p0 + t < n && r < m;
        v[q][t] = (col && rr > t) ? d.vr[r + (int64_t)(p0 + t) * m] : ((col && rr == t) ? T(1) : T(0));
      }
    }
  };
  for (int p0 = 0, it = 0; p0 < n; p0 += JB, ++it) {
    load_v(p0, vc);
    const int buf = it & 1;
    // column `lane` of this panel's T (upper triangular, column-major JB x JB)
    T tcol[JB];
    const T* tp = d.tpan + (int64_t)(p0 / JB) * JB * JB;
#pragma unroll
    for (int q = 0; q < JB; ++q) tcol[q] = (lane < JB && q <= lane) ? tp[q + lane * JB] : T(0);
    double w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) w[i] = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int t = 0; t < JB; ++t)
#pragma unroll
        for (int c = 0; c < NR; ++c) w[t * NR + c] += (double)vc[q][t] * xr[q][c];
    const double s = wave_reduce_scatter<double, K>(w);
    if ((lane & ((1 << SH) - 1)) == 0) red[buf][wv][lane >> SH] = s;
    __syncthreads();
    // u_t = (T^T w)_t on lane t, the reduced w read from LDS as broadcasts
    double u[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      u[c] = 0.0;
#pragma unroll
      for (int q = 0; q < JB; ++q)
        u[c] += (double)tcol[q] *
                (red[buf][0][q * NR + c] + red[buf][1][q * NR + c] + red[buf][2][q * NR + c] + red[buf][3][q * NR + c]);
    }
    // x <- x - V u, u_t broadcast from lane t (uniform, scalar registers)
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      double acc[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) acc[q] = 0.0;
#pragma unroll
      for (int t = 0; t < JB; ++t) {
        const double ut = readlane_d(u[c], t);
#pragma unroll
        for (int q = 0; q < Q; ++q) acc[q] += (double)vc[q][t] * ut;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) xr[q][c] -= acc[q];
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int r = tid + 256 * q;
    if (r < m)
#pragma unroll
      for (int c = 0; c < NR; ++c)
        if (c < nc) x[sl[q] + (int64_t)(c0 + c) * ldx] = xr[q][c];
  }
}

// Dense operators of an interface of at most 64 unknowns (Section 2.8): the
// forward sweep applies U_pp^T (scaling reflectors in order) then Q_pp^T
// (sparsification reflectors in order); the backward sweep applies Q_pp
// (reverse order) then R_pp^{-1}.  mf = Q^T U^T and mb = R^{-1} Q are formed
// by applying those steps to the identity, held in LDS in FP64.  LP adjacent
// lanes share a column (rows part, part + LP, ...): reflector dots reduce
// with log2(LP) lane swaps and no barrier, since a column is only touched by
// its own lanes.
// PM (16, 32 or 64) bounds P; the workgroup has LP PM threads, LP (4, 8 or
// 16) lanes per column.
template <typename T, int PM, int LP>
__global__ void __launch_bounds__(LP * PM) k_iface_form(const ApIface<T>* __restrict__ ds) {
  constexpr int LX = PM + 1;  // padded row stride of X: the row parts of a column fall in distinct banks
  constexpr int NTH = LP * PM;
  static_assert(LP == 4 || LP == 8 || LP == 16, "four, eight or sixteen lanes per column");
  extern __shared__ __align__(16) unsigned char smem[];
  const ApIface<T> d = ds[blockIdx.x];
  const int P = d.P, tid = threadIdx.x, j = tid / LP, part = tid & (LP - 1);
  if (P == 0 || *d.flag != 0) return;
  const int r = *d.rank;
  const bool hasq = r < P;
  double* X = reinterpret_cast<double*>(smem);  // PM x LX
  double* tu = X + PM * LX;                     // PM
  double* tq = tu + PM;                         // PM
  T* vu = reinterpret_cast<T*>(tq + PM);        // P x P column-major
  T* vq = vu + P * P;                           // P x P column-major (first r columns)
  for (int e = tid; e < P * P; e += NTH) {
    vu[e] = d.vru[e];
    vq[e] = (hasq && e < P * r) ? d.vq[e] : T(0);
  }
  if (tid < P) {
    tu[tid] = (double)d.tauu[tid];
    tq[tid] = (hasq && tid < r) ? (double)d.tauq[tid] : 0.0;
  }
  auto ident = [&]() {
    if (j < P)
      for (int q = part; q < P; q += LP) X[q * LX + j] = q == j ? 1.0 : 0.0;
  };
  // X[:, j] <- (I - tau v v^T) X[:, j]; v = column t of V with rows < t zero
  // and, if unit, an implicit 1 at row t
  auto reflect = [&](const T* V, int t, double tau, bool unit) {
    double sdot = 0.0;
    if (j < P)
      for (int q = part; q < P; q += LP) {
        const double v = q < t ? 0.0 : ((q == t && unit) ? 1.0 : (double)V[q + t * P]);
        sdot += v * X[q * LX + j];
      }
    sdot += xshfl<1>(sdot);
    sdot += xshfl<2>(sdot);
    if (LP >= 8) sdot += xshfl<4>(sdot);
    if (LP >= 16) sdot += xshfl<8>(sdot);
    sdot *= tau;
    if (j < P)
      for (int q = part; q < P; q += LP) {
        const double v = q < t ? 0.0 : ((q == t && unit) ? 1.0 : (double)V[q + t * P]);
        X[q * LX + j] -= sdot * v;
      }
  };
  auto store = [&](T* M) {
    if (j < P)
      for (int q = part; q < P; q += LP) M[q + (int64_t)j * P] = (T)X[q * LX + j];
  };
  ident();
  __syncthreads();
  for (int t = 0; t < P; ++t) reflect(vu, t, tu[t], true);
  if (hasq)
    for (int t = 0; t < r; ++t) reflect(vq, t, tq[t], false);
  store(d.mf);
  ident();
  if (hasq)
    for (int t = r - 1; t >= 0; --t) reflect(vq, t, tq[t], false);
  // R^{-1}: R upper triangular on and above the diagonal of vu
  for (int c = P - 1; c >= 0; --c) {
    if (j < P) {
      const double xc = X[c * LX + j] / (double)vu[c + c * P];
      if ((c & (LP - 1)) == part) X[c * LX + j] = xc;
      for (int q = part; q < c; q += LP) X[q * LX + j] -= (double)vu[q + c * P] * xc;
    }
  }
  store(d.mb);
}

// x_p <- M x_p for interfaces of at most 64 unknowns, one wavefront per
// interface (four per workgroup): lane i forms row i, x_j broadcast by
// readlane.  Unscaled interfaces are left alone.
template <typename T>
__global__ void __launch_bounds__(256) k_ap_iface_dense(const ApIface<T>* __restrict__ ds, int64_t n, int backward,
                                                       double* x, int64_t ldx, int nrhs) {
  const int64_t it = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (it >= n) return;
  const ApIface<T> d = ds[it];
  x += d.xoff;
  const int P = d.P, lane = threadIdx.x & 63;
  if (P == 0 || *d.flag != 0) return;
  const T* M = backward ? d.mb : d.mf;
  T mrow[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) mrow[j] = (lane < P && j < P) ? M[lane + (int64_t)j * P] : T(0);
  const int sl = lane < P ? d.slots[lane] : 0;
  for (int c = 0; c < nrhs; ++c) {
    const double xl = lane < P ? x[sl + (int64_t)c * ldx] : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < P) acc += (double)mrow[j] * readlane_d(xl, j);
    if (lane < P) x[sl + (int64_t)c * ldx] = acc;
  }
}

// The same product for launches of few interfaces, where the time is the
// latency of one wavefront: x_p is staged in LDS (per wavefront) and read
// back as broadcasts, and the row dot runs in four independent partial sums
// instead of one chain of readlane-fed FMAs.
template <typename T>
__global__ void __launch_bounds__(256) k_ap_iface_dense_lat(const ApIface<T>* __restrict__ ds, int64_t n,
                                                           int backward, double* x, int64_t ldx, int nrhs) {
  __shared__ double xs[4][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t it = (int64_t)blockIdx.x * 4 + wv;
  if (it >= n) return;
  const ApIface<T> d = ds[it];
  const int P = d.P;
  // the operator's loads are issued before the flag is known (the operators
  // of every interface of at most 64 unknowns are allocated, scaled or not)
  const T* M = backward ? d.mb : d.mf;
  T mrow[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) mrow[j] = (lane < P && j < P) ? M[lane + (int64_t)j * P] : T(0);
  const int sl = lane < P ? d.slots[lane] : 0;
  if (P == 0 || *d.flag != 0) return;
  x += d.xoff;
  for (int c = 0; c < nrhs; ++c) {
    xs[wv][lane] = lane < P ? x[sl + (int64_t)c * ldx] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int j = 0; j < 64; j += 4) {
      a0 += (double)mrow[j] * xs[wv][j];
      a1 += (double)mrow[j + 1] * xs[wv][j + 1];
      a2 += (double)mrow[j + 2] * xs[wv][j + 2];
      a3 += (double)mrow[j + 3] * xs[wv][j + 3];
    }
    // every lane has read xs before the next column overwrites it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < P) x[sl + (int64_t)c * ldx] = (a0 + a1) + (a2 + a3);
  }
}

// Interfaces of at most 64 unknowns, one wavefront each, row `lane` of the
// interface in one lane's registers: forward x_p <- Q^T U^T x_p, backward
// x_p <- R_pp^{-1} Q x_p.  The lane's row of the U/R factor and of the Q
// reflectors is loaded once (independent loads) and reused for every
// reflector and every right-hand side.
template <typename T>
__global__ void __launch_bounds__(64) k_ap_iface_small(const ApIface<T>* __restrict__ ds, double* x, int64_t ldx,
                                                      int nrhs, int backward) {
  const ApIface<T> d = ds[blockIdx.x];
  x += d.xoff;
  const int P = d.P, lane = threadIdx.x;
  if (P == 0 || *d.flag != 0) return;
  const int r = *d.rank;
  const bool hasq = r < P;
  T urow[64], qrow[64];
#pragma unroll
  for (int t = 0; t < 64; ++t) {
    urow[t] = (lane < P && t < P) ? d.vru[lane + (int64_t)t * P] : T(0);
    qrow[t] = (hasq && lane < P && t < r) ? d.vq[lane + (int64_t)t * P] : T(0);
  }
  for (int c = 0; c < nrhs; ++c) {
    double xl = lane < P ? x[d.slots[lane] + (int64_t)c * ldx] : 0.0;
    if (!backward) {
#pragma unroll
      for (int t = 0; t < 64; ++t)
        if (t < P) {
          const double v = lane == t ? 1.0 : (lane > t ? (double)urow[t] : 0.0);
          const double dot = wave_sum(v * xl);
          xl -= (double)d.tauu[t] * dot * v;
        }
#pragma unroll
      for (int t = 0; t < 64; ++t)
        if (hasq && t < r) {
          const double v = (double)qrow[t];
          const double dot = wave_sum(v * xl);
          xl -= (double)d.tauq[t] * dot * v;
        }
    } else {
#pragma unroll
      for (int t = 63; t >= 0; --t)
        if (hasq && t < r) {
          const double v = (double)qrow[t];
          const double dot = wave_sum(v * xl);
          xl -= (double)d.tauq[t] * dot * v;
        }
#pragma unroll
      for (int t = 63; t >= 0; --t)
        if (t < P) {
          if (lane == t) xl = xl / (double)urow[t];
          const double yt = __shfl(xl, t, 64);
          if (lane < t) xl -= (double)urow[t] * yt;
        }
    }
    if (lane < P) x[d.slots[lane] + (int64_t)c * ldx] = xl;
  }
}

__global__ void k_gather_perm(double* xhat, const double* __restrict__ b, int64_t ldb,
                              const int64_t* __restrict__ perm, int64_t N, int nrhs) {
  const int64_t tot = N * nrhs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / N, r = i - c * N;
    xhat[i] = b[perm[r] + c * ldb];
  }
}

// Small integer arrays of several buffers into one (the ranks and error
// flags of every factorization of a batch, so that one copy brings them to
// the host).  One workgroup per operation; the list travels as a kernel
// argument.
constexpr int kIntCopyMax = 64;
struct IntCopyList {
  IntCopy op[kIntCopyMax];
};

__global__ void k_gather_ints(IntCopyList L, int32_t* __restrict__ out) {
  const IntCopy c = L.op[blockIdx.x];
  for (int i = threadIdx.x; i < c.n; i += blockDim.x) out[c.dst + i] = c.src[i];
}

__global__ void k_gather_cols(double* xhat, const double* __restrict__ b, int64_t ldb,
                              const PermCol* __restrict__ pc) {
  const int j = blockIdx.y;
  const PermCol c = pc[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += (int64_t)gridDim.x * blockDim.x)
    xhat[c.xoff + i] = b[c.perm[i] + c.col * ldb];
}

__global__ void k_scatter_cols(double* x, int64_t ldx, const double* __restrict__ xhat,
                               const PermCol* __restrict__ pc) {
  const int j = blockIdx.y;
  const PermCol c = pc[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = c.perm[i];
    x[o + c.col * ldx] = xhat[c.xoff + i] * c.dc[o];
  }
}

__global__ void k_scatter_perm(double* x, int64_t ldx, const double* __restrict__ xhat,
                               const int64_t* __restrict__ perm, const double* __restrict__ dc, int64_t N,
                               int nrhs) {
  const int64_t tot = N * nrhs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / N, r = i - c * N;
    const int64_t o = perm[r];
    x[o + c * ldx] = xhat[i] * dc[o];
  }
}

// dc[j] = 1 / ||A[:, j]||_2 from the CSR values visited in column order
// (csc_idx lists, column by column, the CSR positions of each column's
// entries, so the sum order is fixed).  *zero_col = 1 if a column is zero.
__global__ void k_colnorm(const int64_t* __restrict__ cptr, const int64_t* __restrict__ cidx,
                          const double* __restrict__ val, int64_t n, double* __restrict__ dc, int* zero_col) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t t = cptr[j]; t < cptr[j + 1]; ++t) {
      const double v = val[cidx[t]];
      s += v * v;
    }
    if (s == 0.0) {
      *zero_col = 1;
      dc[j] = 0.0;
    } else {
      dc[j] = 1.0 / sqrt(s);
    }
  }
}

// pool[dst[t]] = val[t] * dc[col[t]]: the pre-scaled matrix scattered into
// the stage-L blocks.
template <typename T>
__global__ void k_scatter_scaled(T* pool, const int64_t* __restrict__ dst, const double* __restrict__ val,
                                 const int32_t* __restrict__ col, const double* __restrict__ dc, int64_t nnz) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x)
    pool[dst[i]] = (T)(val[i] * dc[col[i]]);
}

int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

// Every launcher checks that its kernel was accepted.
static void check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string("launch of ") + what + " failed: " + hipGetErrorString(e));
}

// Largest dynamic LDS a workgroup may use on the current device (bytes).
static size_t device_lds_limit() {
  static const size_t lim = [] {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 * 1024;
    return (size_t)v;
  }();
  return lim;
}

// ------------------------------------------------------------------ launchers
template <typename T>
void launch_copy(const CopyTile<T>* tiles, int64_t ntiles, bool transpose, hipStream_t s) {
  if (ntiles <= 0) return;
  if (transpose) {
    count_launch("k_copy_t");
    hipLaunchKernelGGL(k_copy_t<T>, dim3((unsigned)ntiles), dim3(NT), 0, s, tiles);
    check_launch("k_copy_t");
  } else {
    count_launch("k_copy");
    hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)((ntiles + kCopyTiles - 1) / kCopyTiles)), dim3(NT), 0, s, tiles,
                       ntiles);
    check_launch("k_copy");
  }
}

void launch_zero(const ZeroDesc* d, int64_t n, int64_t blocks, hipStream_t s) {
  if (n <= 0 || blocks <= 0) return;
  count_launch("k_zero");
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, d, n);
  check_launch("k_zero");
}

template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  count_launch("k_fill");
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
  check_launch("k_fill");
}

template <typename T>
void launch_scatter_nz(T* pool, const int64_t* dst, const double* val, int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return;
  count_launch("k_scatter_nz");
  hipLaunchKernelGGL(k_scatter_nz<T>, dim3(grid_for(nnz, 256)), dim3(256), 0, s, pool, dst, val, nnz);
  check_launch("k_scatter_nz");
}

void launch_colnorm(const int64_t* cptr, const int64_t* cidx, const double* val, int64_t n, double* dc,
                    int* zero_col, hipStream_t s) {
  count_launch("k_colnorm");
  hipLaunchKernelGGL(k_colnorm, dim3(grid_for(n, 256)), dim3(256), 0, s, cptr, cidx, val, n, dc, zero_col);
  check_launch("k_colnorm");
}

template <typename T>
void launch_scatter_scaled(T* pool, const int64_t* dst, const double* val, const int32_t* col, const double* dc,
                           int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return;
  count_launch("k_scatter_scaled");
  hipLaunchKernelGGL(k_scatter_scaled<T>, dim3(grid_for(nnz, 256)), dim3(256), 0, s, pool, dst, val, col, dc, nnz);
  check_launch("k_scatter_scaled");
}

static size_t qr_bytes_jb(int max_m, int jb, int eb) {
  const size_t lds = align16((size_t)max_m * (jb + 1) * eb) + align16((size_t)jb * jb * eb) +
                     (size_t)jb * jb * sizeof(double) + 8 * sizeof(double) + (size_t)jb * sizeof(double);
  return lds;
}


// Register-panel QR (k_qr_reg) for matrices of at most NT * Q rows; taller
// ones use the LDS-panel kernel k_qr.  Returns the panel width and Q (0 when
// k_qr is used).
struct QRPlan {
  int jb, q;
};
static QRPlan qr_plan(int max_m, int eb) {
  const int lim = tuning().qr_reg_max_rows;
  if (max_m <= NT) return {16, 1};
  if (max_m <= 2 * NT && lim >= 2 * NT) return {16, 2};
  if (max_m <= 4 * NT && lim >= 4 * NT) return {eb == 8 ? 8 : 16, 4};
  const size_t budget = device_lds_limit();
  for (int jb = 16; jb >= 1; jb >>= 1)
    if (qr_bytes_jb(max_m, jb, eb) <= budget) return {jb, 0};
  return {0, 0};
}

static size_t qr_reg_lds(int max_m, int jb, int eb) { return ((size_t)max_m * jb + (size_t)jb * jb + 10 * jb) * eb; }

// Allow a kernel more than the default 64 KB of dynamic LDS (gfx950: 160 KB
// per workgroup).  Called before every launch that needs it; the attribute
// is set once per kernel.
// The largest size set so far is remembered per kernel, so that a launch
// needing no more makes no runtime call (in particular none while an apply
// is being captured into a graph).
static void allow_lds(const void* fn, size_t bytes, const char* what) {
  if (bytes <= 64 * 1024) return;
  static std::mutex mu;
  static std::map<const void*, size_t> set;
  std::lock_guard<std::mutex> lk(mu);
  auto it = set.find(fn);
  if (it != set.end() && it->second >= bytes) return;
  if (bytes > device_lds_limit()) throw Error(SPAQR_ENOMEM, std::string(what) + ": LDS need exceeds the device limit");
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string(what) + ": cannot raise the LDS limit");
  set[fn] = bytes;
}

int qr_panel_width(int max_m, int eb) { return qr_plan(max_m, eb).jb; }

size_t qr_lds_bytes(int max_m, int jb, int eb) { return qr_bytes_jb(max_m, jb, eb); }

template <typename T>
void launch_qr(const QRDesc<T>* d, int64_t n, int jb, int max_m, hipStream_t s) {
  if (n <= 0) return;
  const QRPlan pl = qr_plan(max_m, sizeof(T));
  if (pl.q > 0 && pl.jb == jb) {
    const size_t lds = qr_reg_lds(max_m, jb, sizeof(T));
#define SPAQR_QRR(J, Q)                                                                      \
  if (jb == J && pl.q == Q) {                                                               \
    allow_lds(reinterpret_cast<const void*>(&k_qr_reg<T, J, Q>), lds, "k_qr_reg");          \
    count_launch("k_qr_reg");                                                              \
    hipLaunchKernelGGL((k_qr_reg<T, J, Q>), dim3((unsigned)n), dim3(NT), lds, s, d);       \
    check_launch("k_qr_reg");                                                               \
    return;                                                                                 \
  }
    if constexpr (sizeof(T) == 4) {
      SPAQR_QRR(16, 1)
      SPAQR_QRR(16, 2)
      SPAQR_QRR(16, 4)
    } else {
      SPAQR_QRR(16, 1)
      SPAQR_QRR(16, 2)
      SPAQR_QRR(8, 4)
    }
#undef SPAQR_QRR
    throw Error(SPAQR_EINVAL, "unsupported register-panel QR shape");
  }
  const size_t lds = qr_bytes_jb(max_m, jb, sizeof(T));
  switch (jb) {
#define SPAQR_QR_CASE(J)                                                   \
  case J:                                                                  \
    allow_lds(reinterpret_cast<const void*>(&k_qr<T, J>), lds, "k_qr");  \
    count_launch("k_qr");                                                     \
    hipLaunchKernelGGL((k_qr<T, J>), dim3((unsigned)n), dim3(NT), lds, s, d); \
    break;
    SPAQR_QR_CASE(1)
    SPAQR_QR_CASE(2)
    SPAQR_QR_CASE(4)
    SPAQR_QR_CASE(8)
    SPAQR_QR_CASE(16)
    SPAQR_QR_CASE(32)
#undef SPAQR_QR_CASE
    default: throw Error(SPAQR_EINVAL, "unsupported QR panel width");
  }
  check_launch("k_qr");
}

static size_t trail_lds(int max_m, int jb, int cw, int eb) {
  return ((size_t)(NT / cw) * jb * cw + 2 * (size_t)jb * cw + (size_t)max_m * (cw + 1)) * eb;
}

template <typename T>
void launch_wy_tblock(const WYBlock<T>* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  count_launch("k_wy_tblock");
  hipLaunchKernelGGL(k_wy_tblock<T>, dim3((unsigned)n), dim3(256), 0, s, d);
  check_launch("k_wy_tblock");
}

template <typename T>
void launch_trail_mfma(const WYTile<T>* d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  count_launch("k_trail_mfma");
  hipLaunchKernelGGL(k_trail_mfma<T>, dim3((unsigned)n), dim3(256), 0, s, d);
  check_launch("k_trail_mfma");
}

int trail_width(int max_m, int eb) {
  const size_t lim = device_lds_limit();
  for (int cw : {16, 8, 4})
    if (trail_lds(max_m, 16, cw, eb) <= lim) return cw;
  return 0;
}

template <typename T>
void launch_trail(const TrailDesc<T>* d, int64_t n, int jb, int cw, int max_m, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = trail_lds(max_m, jb, cw, sizeof(T));
  if (lds > device_lds_limit()) throw Error(SPAQR_ENOMEM, "front too tall for the trailing-update slice");
#define SPAQR_TR(J, W)                                                                      \
  if (jb == J && cw == W) {                                                                \
    allow_lds(reinterpret_cast<const void*>(&k_trail<T, J, W>), lds, "k_trail");          \
    count_launch("k_trail");                                                              \
    hipLaunchKernelGGL((k_trail<T, J, W>), dim3((unsigned)n), dim3(NT), lds, s, d);       \
    check_launch("k_trail");                                                               \
    return;                                                                                \
  }
  SPAQR_TR(16, 16)
  SPAQR_TR(16, 8)
  SPAQR_TR(16, 4)
  SPAQR_TR(8, 16)
  SPAQR_TR(8, 8)
  SPAQR_TR(8, 4)
  SPAQR_TR(4, 16)
  SPAQR_TR(4, 8)
  SPAQR_TR(4, 4)
#undef SPAQR_TR
  throw Error(SPAQR_EINVAL, "unsupported panel width for the trailing update");
}

static size_t scale_small_lds(int max_rows, int max_cols, int jb, int eb) {
  const size_t lb = (size_t)max_cols + 1;
  return ((size_t)max_rows * lb + (size_t)max_rows * (jb + 1) + (size_t)jb * jb +
          std::max(2 * (size_t)jb * max_cols, (size_t)max_cols * lb)) * eb;
}

template <typename T>
void launch_scale_small(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int jb, int max_rows, int max_cols,
                        hipStream_t s) {
  if (n <= 0) return;
  SPAQR_REQUIRE(max_rows <= kScaleSmall && max_cols <= kScaleSmall, SPAQR_EINVAL, "block too large for k_scale_small");
  const size_t lds = scale_small_lds(max_rows, max_cols, jb, sizeof(T));
  switch (jb) {
#define SPAQR_SS_CASE(J)                                                                              \
  case J:                                                                                             \
    allow_lds(reinterpret_cast<const void*>(&k_scale_small<T, J>), lds, "k_scale_small");              \
    count_launch("k_scale_small");                                                                              \
    hipLaunchKernelGGL((k_scale_small<T, J>), dim3((unsigned)n), dim3(NT), lds, s, d, fac, max_rows, max_cols); \
    break;
    SPAQR_SS_CASE(1)
    SPAQR_SS_CASE(2)
    SPAQR_SS_CASE(4)
    SPAQR_SS_CASE(8)
    SPAQR_SS_CASE(16)
    SPAQR_SS_CASE(32)
#undef SPAQR_SS_CASE
    default: throw Error(SPAQR_EINVAL, "unsupported QR panel width");
  }
  check_launch("k_scale_small");
}

template <typename T>
void launch_scale(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int jb, int max_p, int max_rows,
                  int max_cols, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = qr_bytes_jb(max_p, jb, sizeof(T));
  const dim3 grid((unsigned)n, (unsigned)((max_cols + NT - 1) / NT));
  switch (jb) {
#define SPAQR_SC_CASE(J) \
  case J:                                                                                       \
    allow_lds(reinterpret_cast<const void*>(&k_scale<T, J>), lds, "k_scale");                 \
    count_launch("k_scale");                                                                   \
    hipLaunchKernelGGL((k_scale<T, J>), grid, dim3(NT), lds, s, d, fac);                       \
    break;
    SPAQR_SC_CASE(1)
    SPAQR_SC_CASE(2)
    SPAQR_SC_CASE(4)
    SPAQR_SC_CASE(8)
    SPAQR_SC_CASE(16)
    SPAQR_SC_CASE(32)
#undef SPAQR_SC_CASE
    default: throw Error(SPAQR_EINVAL, "unsupported QR panel width");
  }
  check_launch("k_scale");
  launch_scale_right<T>(d, n, fac, max_rows, s);
}

template <typename T>
void launch_scale_right(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int max_rows, hipStream_t s) {
  if (n <= 0) return;
  count_launch("k_scale_right");
  hipLaunchKernelGGL(k_scale_right<T>, dim3((unsigned)n, (unsigned)((max_rows + 15) / 16)), dim3(NT), 0, s, d, fac);
  check_launch("k_scale_right");
}


template <typename T, int PMAX, int NTH>
static void launch_sparsify_small_t(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int max_nb, size_t c_bytes,
                                    hipStream_t s) {
  constexpr int NW = NTH / 64;
  const size_t head = align16(align16((size_t)NW * 8 + 32 + (size_t)NW * 4) + PMAX * sizeof(T) +
                              (size_t)(max_nb + 1) * 4);
  const size_t lim = std::min<size_t>(device_lds_limit(), 64 * 1024);
  size_t cb = std::min(c_bytes, lim > head + 1024 ? lim - head - 512 : 0);
  const int lds_c_elems = (int)(cb / sizeof(T));
  const size_t lds = head + (size_t)lds_c_elems * sizeof(T);
  count_launch("k_sparsify_small");
  hipLaunchKernelGGL((k_sparsify_small<T, PMAX, NTH>), dim3((unsigned)n), dim3(NTH), lds, s, d, nb, lds_c_elems,
                     max_nb);
  check_launch("k_sparsify_small");
}

template <typename T>
void launch_sparsify_small(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int pmax, int max_nb,
                           size_t max_c_elems, hipStream_t s) {
  if (n <= 0) return;
  const size_t cbytes = max_c_elems * sizeof(T);
  // thread counts keep the per-thread column in registers without spills
  // (no FP64 instantiation for 33-64 unknowns is built: those interfaces take
  // the generic kernel)
  constexpr bool F32 = sizeof(T) == 4;
  if (pmax <= 16) {
    launch_sparsify_small_t<T, 16, 1024>(d, n, nb, max_nb, cbytes, s);
  } else if (pmax <= 32) {
    launch_sparsify_small_t<T, 32, F32 ? 1024 : 512>(d, n, nb, max_nb, cbytes, s);
  } else {
    if constexpr (F32) launch_sparsify_small_t<T, 64, 512>(d, n, nb, max_nb, cbytes, s);
    else throw Error(SPAQR_EINVAL, "FP64 interfaces above 32 unknowns use the generic sparsify kernel");
  }
}

template <typename T>
void launch_sparsify(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int max_p, int max_nb, hipStream_t s) {
  if (n <= 0) return;
  const size_t lds = align16((size_t)(max_nb + 1) * sizeof(int)) + (size_t)max_p * sizeof(double) +
                     8 * sizeof(double) + NT * sizeof(double) + NT * sizeof(int);
  count_launch("k_sparsify");
  hipLaunchKernelGGL(k_sparsify<T>, dim3((unsigned)n), dim3(NT), lds, s, d, nb);
  check_launch("k_sparsify");
}

// Register CPQR capacity: P <= PMAX, and the interface's column bound mmax <=
// SP_NT * (CPT + LC) with PMAX * CPT * sizeof(T) / 4 <= 192 registers per
// thread and at most one more column per thread in LDS.  Returns CPT + LC, or
// 0 when the interface does not fit.
static int sp_reg_cap(int eb, int pclass) { return std::min(4, 192 / (pclass * eb / 4)); }

int sparsify_reg_cpt(int eb, int pmax, int mmax) {
  const int pclass = pmax <= 16 ? 16 : (pmax <= 32 ? 32 : 64);
  if (pmax > 64 || (eb == 8 && pclass == 64)) return 0;
  const int cpt = std::max(1, (mmax + SP_NT - 1) / SP_NT);
  const int cap = sp_reg_cap(eb, pclass);
  if (cpt <= cap + 1) return cpt;
  // FP32 interfaces of 33-64 unknowns: one more column per thread in the
  // descriptor's global workspace
  return eb == 4 && pclass == 64 && cpt == cap + 2 ? cpt : 0;
}

bool sparsify_reg_global(int eb, int pmax, int mmax) {
  const int pclass = pmax <= 16 ? 16 : (pmax <= 32 ? 32 : 64);
  const int cpt = sparsify_reg_cpt(eb, pmax, mmax);
  return cpt > 0 && cpt > sp_reg_cap(eb, pclass) + 1;
}

template <typename T>
void launch_sparsify_reg(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int pmax, int mmax, int max_nb,
                         hipStream_t s) {
  if (n <= 0) return;
  const int tot = sparsify_reg_cpt(sizeof(T), pmax, mmax);
  if (tot == 0) throw Error(SPAQR_EINVAL, "interface too large for the register CPQR");
  const int pclass = pmax <= 16 ? 16 : (pmax <= 32 ? 32 : 64);
  const int cap = sp_reg_cap(sizeof(T), pclass);
  const int cpt = std::min(tot, cap), lc = std::min(tot - cpt, 1), gc = tot - cpt - lc;
  constexpr int NW = SP_NT / 64;
  const size_t lds = (size_t)(2 * NW + 1 + lc * SP_NT) * pclass * sizeof(T) + (2 * NW + 2) * sizeof(double) +
                     (size_t)(2 * NW + max_nb + 1) * sizeof(int);
#define SPAQR_SPR(PM, CP, L, G)                                                                           \
  if (pclass == PM && cpt == CP && lc == L && gc == G) {                                                 \
    allow_lds(reinterpret_cast<const void*>(&k_cpqr_reg<T, PM, CP, L, G>), lds, "k_cpqr_reg");          \
    count_launch("k_cpqr_reg");                                                                               \
    hipLaunchKernelGGL((k_cpqr_reg<T, PM, CP, L, G>), dim3((unsigned)n), dim3(SP_NT), lds, s, d, nb, max_nb); \
    check_launch("k_cpqr_reg");                                                                          \
    return;                                                                                              \
  }
  if constexpr (sizeof(T) == 4) {
    SPAQR_SPR(16, 1, 0, 0)
    SPAQR_SPR(16, 2, 0, 0)
    SPAQR_SPR(16, 3, 0, 0)
    SPAQR_SPR(16, 4, 0, 0)
    SPAQR_SPR(16, 4, 1, 0)
    SPAQR_SPR(32, 1, 0, 0)
    SPAQR_SPR(32, 2, 0, 0)
    SPAQR_SPR(32, 3, 0, 0)
    SPAQR_SPR(32, 4, 0, 0)
    SPAQR_SPR(32, 4, 1, 0)
    SPAQR_SPR(64, 1, 0, 0)
    SPAQR_SPR(64, 2, 0, 0)
    SPAQR_SPR(64, 3, 0, 0)
    SPAQR_SPR(64, 3, 1, 0)
    SPAQR_SPR(64, 3, 1, 1)
  } else {
    SPAQR_SPR(16, 1, 0, 0)
    SPAQR_SPR(16, 2, 0, 0)
    SPAQR_SPR(16, 3, 0, 0)
    SPAQR_SPR(16, 4, 0, 0)
    SPAQR_SPR(16, 4, 1, 0)
    SPAQR_SPR(32, 1, 0, 0)
    SPAQR_SPR(32, 2, 0, 0)
    SPAQR_SPR(32, 3, 0, 0)
    SPAQR_SPR(32, 3, 1, 0)
  }
#undef SPAQR_SPR
  throw Error(SPAQR_EINVAL, "unsupported register CPQR shape");
}

static size_t coop_lds(int max_p, int max_nb, int eb, int cpt, bool lc) {
  return (size_t)((max_p + 3) & ~3) * eb + (lc ? (size_t)max_p * 64 * cpt * eb : 0) +
         (size_t)(max_nb + 1) * sizeof(int);
}

// columns stay in LDS when a workgroup's slice fits in 144 KB
static bool coop_in_lds(int max_p, int cpt, int eb) { return (size_t)max_p * 64 * cpt * eb <= (size_t)144 * 1024; }

template <typename T, int CPT, bool LC>
static const void* coop_fn() {
  return reinterpret_cast<const void*>(&k_cpqr_coop<T, CPT, LC>);
}

template <typename T>
static const void* coop_kernel(int cpt, bool lc) {
  switch (cpt) {
    case 1: return lc ? coop_fn<T, 1, true>() : coop_fn<T, 1, false>();
    case 2: return lc ? coop_fn<T, 2, true>() : coop_fn<T, 2, false>();
    case 4: return lc ? coop_fn<T, 4, true>() : coop_fn<T, 4, false>();
    case 8: return lc ? coop_fn<T, 8, true>() : coop_fn<T, 8, false>();
    default: return nullptr;
  }
}

template <typename T>
int sparsify_coop_capacity(int cpt, int max_p, int max_nb) {
  const bool lc = coop_in_lds(max_p, cpt, sizeof(T));
  const void* fn = coop_kernel<T>(cpt, lc);
  if (!fn) return 0;
  const size_t lds = coop_lds(max_p, max_nb, sizeof(T), cpt, lc);
  int per_cu = 0, dev = 0, cus = 0;
  if (lds > 160 * 1024) return 0;
  allow_lds(fn, lds, "k_cpqr_coop");
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess) return 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

template <typename T>
bool launch_sparsify_coop(const SpDesc<T>* d, const CoopItem* items, int nitems, int total_blocks, int cpt,
                          const SpNbr* nb, int max_p, int max_nb, double* ckey, int* cpos, T* ccol, int* done,
                          int kmax_all, hipStream_t s) {
  if (nitems <= 0) return true;
  if (total_blocks > sparsify_coop_capacity<T>(cpt, max_p, max_nb)) return false;
  const bool lc = coop_in_lds(max_p, cpt, sizeof(T));
  const size_t lds = coop_lds(max_p, max_nb, sizeof(T), cpt, lc);
  void* args[] = {(void*)&d, (void*)&nb, (void*)&items, (void*)&nitems, (void*)&total_blocks, (void*)&max_p,
                  (void*)&max_nb, (void*)&ckey, (void*)&cpos, (void*)&ccol, (void*)&done, (void*)&kmax_all};
  const void* fn = coop_kernel<T>(cpt, lc);
  if (!fn) throw Error(SPAQR_EINVAL, "unsupported columns per thread in the cooperative CPQR");
  count_launch("k_cpqr_coop");
  const hipError_t e = hipLaunchCooperativeKernel(fn, dim3((unsigned)total_blocks), dim3(64), args, lds, s);
  if (e != hipSuccess)
    throw Error(SPAQR_EDEVICE, std::string("cooperative launch of k_cpqr_coop failed: ") + hipGetErrorString(e));
  return true;
}

// FP64 rows an apply workgroup may stage in LDS: up to the device's limit
// per workgroup (160 KB on gfx950), less room for the small work arrays.
static size_t apply_lds_budget() { return device_lds_limit() - 2048; }

int apply_rhs_block(int max_rows, int nrhs) {
  const size_t lim = apply_lds_budget();
  int rb = RBMAX;
  if (rb > nrhs) rb = nrhs;
  while (rb > 1 && (size_t)max_rows * rb * sizeof(double) > lim) --rb;
  if ((size_t)max_rows * rb * sizeof(double) > lim) return 0;
  return rb;
}

#define SPAQR_AP_LAUNCH(KERNEL, DESC)                                                           \
  template <typename T>                                                                         \
  void launch_##KERNEL(const DESC<T>* d, int64_t n, int max_rows, double* x, int64_t ldx, int nrhs, \
                       hipStream_t s) {                                                         \
    if (n <= 0 || nrhs <= 0) return;                                                            \
    const int rb = apply_rhs_block(max_rows, nrhs);                                             \
    if (rb < 1) throw Error(SPAQR_ENOMEM, "apply: item too large for LDS");                     \
    const size_t lds = (size_t)max_rows * rb * sizeof(double);                                  \
    allow_lds(reinterpret_cast<const void*>(&k_ap_##KERNEL<T>), lds, "k_ap_" #KERNEL);         \
    count_launch("k_ap_" #KERNEL);                                                              \
    hipLaunchKernelGGL(k_ap_##KERNEL<T>, dim3((unsigned)n, (unsigned)((nrhs + rb - 1) / rb)),  \
                       dim3(64), lds, s, d, x, ldx, nrhs, rb);                                  \
    check_launch("k_ap_" #KERNEL);                                                              \
  }
SPAQR_AP_LAUNCH(front_fwd, ApFront)
SPAQR_AP_LAUNCH(front_bwd, ApFront)
SPAQR_AP_LAUNCH(iface_fwd, ApIface)
SPAQR_AP_LAUNCH(iface_bwd, ApIface)
#undef SPAQR_AP_LAUNCH

template <typename T>
void launch_front_fwd_wy(const ApFront<T>* d, int64_t n, int jb, int max_rows, double* x, int64_t ldx, int nrhs,
                         hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  if ((jb == 16 || jb == 8) && max_rows <= 1024) {
    const int q = max_rows <= 256 ? 1 : (max_rows <= 512 ? 2 : 4);
    const int nr = nrhs == 1 ? 1 : (nrhs == 2 || jb == 16 ? 2 : 4);
    const dim3 grid((unsigned)n, (unsigned)((nrhs + nr - 1) / nr));
#define SPAQR_FWR(J, Q, R)                                                                             \
  if (jb == J && q == Q && nr == R) {                                                                  \
    count_launch("k_ap_front_fwd_reg");                                                                \
    hipLaunchKernelGGL((k_ap_front_fwd_reg<T, J, Q, R>), grid, dim3(256), 0, s, d, x, ldx, nrhs);      \
    check_launch("k_ap_front_fwd_reg");                                                               \
    return;                                                                                           \
  }
    SPAQR_FWR(16, 1, 1)
    SPAQR_FWR(16, 2, 1)
    SPAQR_FWR(16, 4, 1)
    SPAQR_FWR(16, 1, 2)
    SPAQR_FWR(16, 2, 2)
    SPAQR_FWR(16, 4, 2)
    SPAQR_FWR(8, 1, 1)
    SPAQR_FWR(8, 2, 1)
    SPAQR_FWR(8, 4, 1)
    SPAQR_FWR(8, 1, 2)
    SPAQR_FWR(8, 2, 2)
    SPAQR_FWR(8, 4, 2)
    SPAQR_FWR(8, 1, 4)
    SPAQR_FWR(8, 2, 4)
    SPAQR_FWR(8, 4, 4)
#undef SPAQR_FWR
  }
  const int rb = apply_rhs_block(max_rows + 1, nrhs);
  if (rb < 1) throw Error(SPAQR_ENOMEM, "apply: front too large for LDS");
  const size_t lds = ((size_t)max_rows * rb + 6 * 32) * sizeof(double);
  const dim3 grid((unsigned)n, (unsigned)((nrhs + rb - 1) / rb));
  switch (jb) {
#define SPAQR_FW_CASE(J) \
  case J:                                                                                  \
    allow_lds(reinterpret_cast<const void*>(&k_ap_front_fwd_wy<T, J>), lds, "k_ap_front_fwd_wy"); \
    count_launch("k_ap_front_fwd_wy");                                                           \
    hipLaunchKernelGGL((k_ap_front_fwd_wy<T, J>), grid, dim3(256), lds, s, d, x, ldx, nrhs, rb); \
    break;
    SPAQR_FW_CASE(1)
    SPAQR_FW_CASE(2)
    SPAQR_FW_CASE(4)
    SPAQR_FW_CASE(8)
    SPAQR_FW_CASE(16)
    SPAQR_FW_CASE(32)
#undef SPAQR_FW_CASE
    default: throw Error(SPAQR_EINVAL, "unsupported panel width in the apply");
  }
  check_launch("k_ap_front_fwd_wy");
}

template <typename T>
void launch_front_bwd_reg(const ApFront<T>* d, int64_t n, int max_n, int max_k, double* x, int64_t ldx, int nrhs,
                          hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  // LDS, sized for the launch's fronts (occupancy): y_s and a chunk of x_j
  // (rb columns each), 256 partial sums, the R_ss tile (the rows above a
  // 64-row diagonal block are at most max_n - 64)
  const int chunk = std::max(1, std::min(kBwdChunk, (max_k + 63) / 64 * 64));
  const int tile_rows = max_n - 64 > 64 ? kBwdTile : 64;
  const size_t tile = (size_t)tile_rows * 65 * sizeof(T) + 256 * sizeof(double);
  const size_t lim = apply_lds_budget() - tile;
  const size_t per_rhs = (size_t)(max_n + chunk) * sizeof(double);
  int rb = std::min(RBMAX, nrhs);
  while (rb > 1 && per_rhs * rb > lim) --rb;
  if (per_rhs * rb > lim) throw Error(SPAQR_ENOMEM, "apply: front too large for LDS");
  const size_t lds = per_rhs * rb + tile;
  allow_lds(reinterpret_cast<const void*>(&k_ap_front_bwd_reg<T>), lds, "k_ap_front_bwd_reg");
  count_launch("k_ap_front_bwd_reg");
  hipLaunchKernelGGL(k_ap_front_bwd_reg<T>, dim3((unsigned)n, (unsigned)((nrhs + rb - 1) / rb)), dim3(256), lds, s,
                     d, x, ldx, nrhs, rb, chunk, tile_rows);
  check_launch("k_ap_front_bwd_reg");
}

template <typename T, int PM>
static void launch_iface_form_t(const ApIface<T>* d, int64_t n, hipStream_t s) {
  // more lanes per column than four: shorter chains per reflector where the
  // LDS limits the workgroups per CU
  constexpr int LP = PM >= 64 ? 16 : 8;
  const size_t lds = ((size_t)PM * (PM + 1) + 2 * PM) * sizeof(double) + 2 * (size_t)PM * PM * sizeof(T);
  allow_lds(reinterpret_cast<const void*>(&k_iface_form<T, PM, LP>), lds, "k_iface_form");
  count_launch("k_iface_form");
  hipLaunchKernelGGL((k_iface_form<T, PM, LP>), dim3((unsigned)n), dim3(LP * PM), lds, s, d);
  check_launch("k_iface_form");
}

template <typename T>
void launch_iface_form(const ApIface<T>* d, int64_t n, int max_p, hipStream_t s) {
  if (n <= 0) return;
  SPAQR_REQUIRE(max_p <= 64, SPAQR_EINVAL, "dense interface operators need P <= 64");
  if (max_p <= 16) launch_iface_form_t<T, 16>(d, n, s);
  else if (max_p <= 32) launch_iface_form_t<T, 32>(d, n, s);
  else launch_iface_form_t<T, 64>(d, n, s);
}

template <typename T>
void launch_iface_dense(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                        hipStream_t s, int max_p) {
  if (n <= 0 || nrhs <= 0) return;
  if (max_p > 64) {
    launch_iface_dense_big<T>(d, n, backward, x, ldx, nrhs, s);
    return;
  }
  // up to 2048 interfaces the LDS-broadcast kernel is faster (measured: 9 us
  // against 20 us for one to a few hundred interfaces of 64 unknowns); beyond,
  // the readlane kernel keeps more loads in flight
  if (n <= 2048) {
    count_launch("k_ap_iface_dense");
    hipLaunchKernelGGL(k_ap_iface_dense_lat<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, d, n,
                       backward ? 1 : 0, x, ldx, nrhs);
    check_launch("k_ap_iface_dense");
    return;
  }
  count_launch("k_ap_iface_dense");
  hipLaunchKernelGGL(k_ap_iface_dense<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, d, n, backward ? 1 : 0, x,
                     ldx, nrhs);
  check_launch("k_ap_iface_dense");
}

template <typename T>
void launch_iface_small(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                        hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  count_launch("k_ap_iface_small");
  hipLaunchKernelGGL(k_ap_iface_small<T>, dim3((unsigned)n), dim3(64), 0, s, d, x, ldx, nrhs, backward ? 1 : 0);
  check_launch("k_ap_iface_small");
}

void launch_gather_perm(double* xhat, const double* b, int64_t ldb, const int64_t* perm, int64_t N,
                        int nrhs, hipStream_t s) {
  count_launch("k_gather_perm");
  hipLaunchKernelGGL(k_gather_perm, dim3(grid_for(N * nrhs, 256)), dim3(256), 0, s, xhat, b, ldb, perm,
                     N, nrhs);
  check_launch("k_gather_perm");
}

void launch_gather_cols(double* xhat, const double* b, int64_t ldb, const PermCol* pc, int ncols, int64_t max_n,
                        hipStream_t s) {
  if (ncols <= 0 || max_n <= 0) return;
  const unsigned gxn = (unsigned)std::min<int64_t>(1024, (max_n + 255) / 256);
  count_launch("k_gather_cols");
  hipLaunchKernelGGL(k_gather_cols, dim3(gxn, (unsigned)ncols), dim3(256), 0, s, xhat, b, ldb, pc);
  check_launch("k_gather_cols");
}

void launch_gather_ints(const IntCopy* ops, int nops, int32_t* out, hipStream_t s) {
  for (int i0 = 0; i0 < nops; i0 += kIntCopyMax) {
    IntCopyList L{};
    const int n = std::min(kIntCopyMax, nops - i0);
    for (int i = 0; i < n; ++i) L.op[i] = ops[i0 + i];
    count_launch("k_gather_ints");
    hipLaunchKernelGGL(k_gather_ints, dim3((unsigned)n), dim3(256), 0, s, L, out);
    check_launch("k_gather_ints");
  }
}

void launch_scatter_cols(double* x, int64_t ldx, const double* xhat, const PermCol* pc, int ncols, int64_t max_n,
                         hipStream_t s) {
  if (ncols <= 0 || max_n <= 0) return;
  const unsigned gxn = (unsigned)std::min<int64_t>(1024, (max_n + 255) / 256);
  count_launch("k_scatter_cols");
  hipLaunchKernelGGL(k_scatter_cols, dim3(gxn, (unsigned)ncols), dim3(256), 0, s, x, ldx, xhat, pc);
  check_launch("k_scatter_cols");
}

void launch_scatter_perm(double* x, int64_t ldx, const double* xhat, const int64_t* perm,
                         const double* dc, int64_t N, int nrhs, hipStream_t s) {
  count_launch("k_scatter_perm");
  hipLaunchKernelGGL(k_scatter_perm, dim3(grid_for(N * nrhs, 256)), dim3(256), 0, s, x, ldx, xhat, perm,
                     dc, N, nrhs);
  check_launch("k_scatter_perm");
}

#define SPAQR_INST(T)                                                                                  \
  template void launch_copy<T>(const CopyTile<T>*, int64_t, bool, hipStream_t);                       \
  template void launch_fill<T>(T*, int64_t, T, hipStream_t);                                          \
  template void launch_scatter_nz<T>(T*, const int64_t*, const double*, int64_t, hipStream_t);       \
  template void launch_scatter_scaled<T>(T*, const int64_t*, const double*, const int32_t*, const double*, \
                                         int64_t, hipStream_t);                                      \
  template void launch_qr<T>(const QRDesc<T>*, int64_t, int, int, hipStream_t);                      \
  template void launch_trail<T>(const TrailDesc<T>*, int64_t, int, int, int, hipStream_t);           \
  template void launch_wy_tblock<T>(const WYBlock<T>*, int64_t, hipStream_t);                          \
  template void launch_trail_mfma<T>(const WYTile<T>*, int64_t, hipStream_t);                          \
  template void launch_scale<T>(const ScaleBlk<T>*, int64_t, const ScaleFac<T>*, int, int, int, int, hipStream_t);                                                                      \
  template void launch_scale_right<T>(const ScaleBlk<T>*, int64_t, const ScaleFac<T>*, int, hipStream_t);                                                                      \
  template void launch_scale_small<T>(const ScaleBlk<T>*, int64_t, const ScaleFac<T>*, int, int, int, hipStream_t); \
  template void launch_sparsify<T>(const SpDesc<T>*, int64_t, const SpNbr*, int, int, hipStream_t); \
  template void launch_sparsify_small<T>(const SpDesc<T>*, int64_t, const SpNbr*, int, int, size_t, hipStream_t); \
  template void launch_sparsify_reg<T>(const SpDesc<T>*, int64_t, const SpNbr*, int, int, int, hipStream_t); \
  template void launch_front_fwd<T>(const ApFront<T>*, int64_t, int, double*, int64_t, int, hipStream_t); \
  template void launch_front_bwd<T>(const ApFront<T>*, int64_t, int, double*, int64_t, int, hipStream_t); \
  template void launch_iface_fwd<T>(const ApIface<T>*, int64_t, int, double*, int64_t, int, hipStream_t); \
  template void launch_iface_bwd<T>(const ApIface<T>*, int64_t, int, double*, int64_t, int, hipStream_t); \
  template void launch_front_fwd_wy<T>(const ApFront<T>*, int64_t, int, int, double*, int64_t, int, hipStream_t); \
  template void launch_front_bwd_reg<T>(const ApFront<T>*, int64_t, int, int, double*, int64_t, int, hipStream_t); \
  template void launch_iface_small<T>(const ApIface<T>*, int64_t, bool, double*, int64_t, int, hipStream_t); \
  template void launch_iface_form<T>(const ApIface<T>*, int64_t, int, hipStream_t);                  \
  template int sparsify_coop_capacity<T>(int, int, int);                                               \
  template bool launch_sparsify_coop<T>(const SpDesc<T>*, const CoopItem*, int, int, int, const SpNbr*, int, int, \
                                        double*, int*, T*, int*, int, hipStream_t);                    \
  template void launch_iface_dense<T>(const ApIface<T>*, int64_t, bool, double*, int64_t, int, hipStream_t, int);
SPAQR_INST(float)
SPAQR_INST(double)
#undef SPAQR_INST
template void launch_fill<int>(int*, int64_t, int, hipStream_t);

}  // namespace spaqr
