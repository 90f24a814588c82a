// Sparsification of interfaces without block-diagonal scaling (Section 2.5,
// Lemma 1), one workgroup per interface, FP64 arithmetic on the blocks of
// the factorization's precision.
//
// For an interface p with row neighbours n_r (blocks (i, p)) and column
// neighbours n_c (blocks (p, j)), each at its current size:
//
//   1. sigma = 1 / sigma_min(A_p), A_p = [A_pp; A_np]: Golub-Kahan
//      bidiagonalization of A_p by Householder reflectors from both sides,
//      then bisection on the Golub-Kahan tridiagonal of the bidiagonal (zero
//      diagonal, off-diagonals d_0, e_0, d_1, ...; its eigenvalues are the
//      +-sigma_i), 65-way per round, one Sturm count per lane of a wavefront;
//   2. C = [A_np^T | sigma A_pp^T A_pn] (P x m);
//   3. partial column-pivoted QR of C with exact column norms at every step,
//      first maximum as the pivot, stopped by |R_kk| < eps |R_11|; rank r.
//      If r = P nothing is dropped and p is left alone (as if its sigma_min
//      were zero): the blocks are untouched and the interface's operators are
//      the identity;
//   4. A_ip <- A_ip Q restricted to its first r columns (the rows of W);
//   5. A_pp Q; Householder QR of its last f = P - r columns gives H and
//      R_ff; H^T on the first r columns gives [R_fc; A_cc], on A_pn gives
//      [R_fn; A_cn] (R_fn, of norm O(eps) by Lemma 1, is dropped); the last r
//      rows become the new rows of p, stored first;
//   6. the dense operators of the apply: forward M_f = Pi H^T (Pi moves the
//      last r rows to the front), backward M_b = Q T with
//      T = [[I_r, 0], [-R_ff^{-1} R_fc, R_ff^{-1}]] (the right factor
//      R_f^{-1} in the coarse-first column order).
//
// Every step is the plain BLAS-2 form, each reflector applied by the whole
// workgroup (a wavefront per column where columns are contiguous, a thread
// per row or per column otherwise), in a per-interface FP64 workspace in
// global memory.  Interfaces of one colour are independent (they share no
// block); colours run in stream order.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>
#include <string>

#include "common.hpp"
#include "kernels.hpp"
#include "profile.hpp"

namespace spaqr {

namespace {

// threads per workgroup: 256 for launches of more than 512 interfaces of at
// most 64 unknowns, 1024 otherwise (more wavefronts in flight per reflector)
constexpr int kNTSmall = 256, kNTWide = 1024;

__device__ __forceinline__ double u_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// workgroup sum, returned to every thread (deterministic order)
template <int NT>
__device__ double u_wg_sum(double v, double* red) {
  v = u_wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) s += red[q];
  return s;
}

// largest value, lowest index among equal values, returned to every thread
template <int NT>
__device__ void u_wg_argmax(double& v, int& i, double* sv, int* si) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(i, o, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = v;
    si[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int q = 1; q < NT / 64; ++q)
    if (sv[q] > v || (sv[q] == v && si[q] < i)) {
      v = sv[q];
      i = si[q];
    }
}

// Householder reflector of x[0], x[inc], ..., x[(n-1) inc] in the xLARFG
// convention: beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta,
// v = [1, x_tail / (alpha - beta)].  x[0] <- beta, the tail <- v[1:]; a zero
// tail gives tau = 0 and leaves x unchanged.
template <int NT>
__device__ double u_larfg(double* x, int n, int64_t inc, double* red) {
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = 1 + t; i < n; i += NT) {
    const double v = x[i * inc];
    s += v * v;
  }
  s = u_wg_sum<NT>(s, red);
  const double alpha = x[0];
  if (s == 0.0) return 0.0;
  const double beta = -copysign(hypot(alpha, sqrt(s)), alpha);
  const double den = alpha - beta;
  __syncthreads();  // alpha read by every thread before x[0] changes
  for (int i = 1 + t; i < n; i += NT) x[i * inc] /= den;
  if (t == 0) x[0] = beta;
  __syncthreads();
  return (beta - alpha) / beta;
}

// A[0:n, j] -= tau v (v^T A[0:n, j]) for the ncols columns of a column-major
// A (leading dimension lda), v[0] = 1, v[i] = vv[i]; a wavefront per column.
// v never overlaps the columns it is applied to.
template <int NT>
__device__ void u_left(const double* __restrict__ vv, int n, double tau, double* __restrict__ A, int64_t lda,
                       int ncols) {
  if (tau != 0.0) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int j = w; j < ncols; j += NT / 64) {
      double* __restrict__ a = A + j * lda;
      double s0 = 0.0, s1 = 0.0;
      int i = l;
      for (; i + 64 < n; i += 128) {
        s0 += (i == 0 ? 1.0 : vv[i]) * a[i];
        s1 += vv[i + 64] * a[i + 64];
      }
      if (i < n) s0 += (i == 0 ? 1.0 : vv[i]) * a[i];
      const double s = u_wave_sum(s0 + s1) * tau;
#pragma unroll 4
      for (int q = l; q < n; q += 64) a[q] -= (q == 0 ? 1.0 : vv[q]) * s;
    }
  }
  __syncthreads();
}

// The same reflector on three column-major blocks with one leading dimension
// (n0, n1 and n2 columns of A0, A1, A2) in one pass: one barrier, and the
// wavefronts share out all n0 + n1 + n2 columns.
template <int NT>
__device__ void u_left3(const double* __restrict__ vv, int n, double tau, int64_t lda, double* __restrict__ A0,
                        int n0, double* __restrict__ A1, int n1, double* __restrict__ A2, int n2) {
  if (tau != 0.0) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int j = w; j < n0 + n1 + n2; j += NT / 64) {
      double* __restrict__ a = j < n0 ? A0 + j * lda : (j < n0 + n1 ? A1 + (j - n0) * lda : A2 + (j - n0 - n1) * lda);
      double s0 = 0.0, s1 = 0.0;
      int i = l;
      for (; i + 64 < n; i += 128) {
        s0 += (i == 0 ? 1.0 : vv[i]) * a[i];
        s1 += vv[i + 64] * a[i + 64];
      }
      if (i < n) s0 += (i == 0 ? 1.0 : vv[i]) * a[i];
      const double s = u_wave_sum(s0 + s1) * tau;
#pragma unroll 4
      for (int q = l; q < n; q += 64) a[q] -= (q == 0 ? 1.0 : vv[q]) * s;
    }
  }
  __syncthreads();
}

// A[i, 0:n] -= tau (A[i, 0:n] v) v^T for the nrows rows of a column-major A,
// v (v[0] = 1) in LDS; a thread per row.
template <int NT>
__device__ void u_right(const double* __restrict__ v, int n, double tau, double* __restrict__ A, int64_t lda,
                        int nrows) {
  if (tau != 0.0) {
    for (int i = threadIdx.x; i < nrows; i += NT) {
      double s0 = 0.0, s1 = 0.0;
      int q = 0;
      for (; q + 1 < n; q += 2) {
        s0 += A[i + q * lda] * v[q];
        s1 += A[i + (q + 1) * lda] * v[q + 1];
      }
      if (q < n) s0 += A[i + q * lda] * v[q];
      const double s = (s0 + s1) * tau;
#pragma unroll 4
      for (int u = 0; u < n; ++u) A[i + u * lda] -= s * v[u];
    }
  }
  __syncthreads();
}

// number of eigenvalues below x of the 2n x 2n tridiagonal with zero
// diagonal and off-diagonals d_0, e_0, d_1, e_1, ..., d_{n-1} (Sturm count
// of the LDL^T recurrence, pivots kept away from zero by pivmin)
__device__ int u_tgk_count(const double* d, const double* e, int n, double x, double pivmin) {
  double q = -x;
  int cnt = q < 0.0 ? 1 : 0;
  for (int t = 1; t < 2 * n; ++t) {
    const double b = (t & 1) ? d[t >> 1] : e[(t >> 1) - 1];
    q = -x - b * b / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0 ? 1 : 0;
  }
  return cnt;
}

// smallest singular value of the upper bidiagonal (d, e) by multisection on
// its Golub-Kahan tridiagonal (eigenvalues -sigma_i, +sigma_i): the smallest
// x > 0 with at least n + 1 eigenvalues below it.  Called by one wavefront;
// every lane returns the result.
__device__ double u_bidiag_smin(const double* d, const double* e, int n) {
  const int lane = threadIdx.x & 63;
  double hi = 0.0, bmax = 0.0, dmin = INFINITY;
  for (int t = 0; t < 2 * n - 1; ++t) {
    const double b = fabs((t & 1) ? e[t >> 1] : d[t >> 1]);
    const double bn = t + 1 < 2 * n - 1 ? fabs(((t + 1) & 1) ? e[(t + 1) >> 1] : d[(t + 1) >> 1]) : 0.0;
    hi = fmax(hi, b + bn);
    bmax = fmax(bmax, b);
  }
  if (n >= 1) hi = fmax(hi, fabs(d[0]));
  for (int t = 0; t < n; ++t) dmin = fmin(dmin, fabs(d[t]));
  if (hi == 0.0 || dmin == 0.0) return 0.0;  // a zero diagonal entry: singular
  const double pivmin = DBL_MIN * fmax(1.0, bmax * bmax);
  double lo = 0.0;
  hi = hi * (1.0 + 8.0 * DBL_EPSILON);
  for (int round = 0; round < 64; ++round) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const bool ge = u_tgk_count(d, e, n, x, pivmin) >= n + 1;
    const unsigned long long bal = __ballot(ge);
    if (bal == 0ull) {
      lo = __shfl(x, 63, 64);
    } else {
      const int j = __ffsll((long long)bal) - 1;
      const double xj = __shfl(x, j, 64);
      const double xl = __shfl(x, j > 0 ? j - 1 : 0, 64);
      if (j > 0) lo = xl;
      hi = xj;
    }
    if (hi - lo <= 2.0 * DBL_EPSILON * hi) break;
  }
  return 0.5 * (lo + hi);
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_sparsify_unscaled(const SpuDesc<T>* __restrict__ ds,
                                                         const SpNbr* __restrict__ nbs) {
  __shared__ double red[NT / 64];
  __shared__ double sv[NT / 64];
  __shared__ int si[NT / 64];
  __shared__ double vbuf[kSpuMaxP];
  __shared__ int s_w[kSpuMaxNbr], s_off[kSpuMaxNbr + 1];
  __shared__ double s_smin;
  const SpuDesc<T> d = ds[blockIdx.x];
  const int t = threadIdx.x;
  const int P = d.P;
  if (P == 0) return;
  const int nn = d.nrow + d.ncol;
  const SpNbr* nb = nbs + d.nb;
  // current sizes of the neighbours (those of earlier colours were sparsified)
  for (int q = t; q < nn; q += NT) s_w[q] = d.rank[nb[q].cluster];
  __syncthreads();
  if (t == 0) {
    int o = 0;
    for (int q = 0; q < nn; ++q) {
      s_off[q] = o;
      o += s_w[q];
    }
    s_off[nn] = o;
  }
  __syncthreads();
  const int mr = s_off[d.nrow], m = s_off[nn], mc = m - mr;
  const int64_t MR = d.mr_max, MC = d.mc_max, M = MR + MC;
  double* G = d.ws;  // (P + MR) x P, column-major
  const int64_t ldg = P + MR;
  double* Cw = G + ldg * P;        // P x M, row-major
  double* B = Cw + (int64_t)P * M;  // P x P, column-major
  double* N = B + (int64_t)P * P;   // P x MC, column-major
  double* E = N + (int64_t)P * MC;  // P x P, column-major
  double* Vq = E + (int64_t)P * P;  // P x P, column-major
  double* tq = Vq + (int64_t)P * P;
  double* tH = tq + P;
  double* dd = tH + P;
  double* ee = dd + P;
  int* perm = reinterpret_cast<int*>(ee + P);
  int* iperm = perm + M;
  T* pool = d.pool;
  T* app = pool + d.app;
  const int mrows = P + mr;

  // ---- gather A_p (G), A_pp (B) and A_pn (N)
  for (int e = t; e < P * P; e += NT) {
    const int a = e / P, c = e - a * P;
    const double v = (double)app[e];
    G[a + c * ldg] = v;
    B[a + (int64_t)c * P] = v;
  }
  for (int q = 0; q < d.nrow; ++q) {
    const T* blk = pool + nb[q].blk;
    const int w = s_w[q], ld = nb[q].ld, o = s_off[q];
    for (int e = t; e < w * P; e += NT) {
      const int a = e / P, c = e - a * P;
      G[(P + o + a) + c * ldg] = (double)blk[(int64_t)a * ld + c];
    }
  }
  for (int q = d.nrow; q < nn; ++q) {
    const T* blk = pool + nb[q].blk;
    const int w = s_w[q], ld = nb[q].ld, o = s_off[q] - mr;
    for (int e = t; e < P * w; e += NT) {
      const int a = e / w, c = e - a * w;
      N[a + (int64_t)(o + c) * P] = (double)blk[(int64_t)a * ld + c];
    }
  }
  __syncthreads();

  // ---- Golub-Kahan bidiagonalization of A_p (mrows >= P)
  for (int k = 0; k < P; ++k) {
    double* gk = G + k + (int64_t)k * ldg;
    const double tl = u_larfg<NT>(gk, mrows - k, 1, red);
    if (t == 0) dd[k] = gk[0];
    u_left<NT>(gk, mrows - k, tl, gk + ldg, ldg, P - k - 1);
    if (k + 1 < P) {
      double* rk = G + k + (int64_t)(k + 1) * ldg;
      const double tr = u_larfg<NT>(rk, P - k - 1, ldg, red);
      if (t == 0) ee[k] = rk[0];
      for (int u = t; u < P - k - 1; u += NT) vbuf[u] = u == 0 ? 1.0 : rk[(int64_t)u * ldg];
      __syncthreads();
      u_right<NT>(vbuf, P - k - 1, tr, G + (k + 1) + (int64_t)(k + 1) * ldg, ldg, mrows - k - 1);
    }
  }
  __syncthreads();
  if (t < 64) {
    const double smin = u_bidiag_smin(dd, ee, P);
    if (t == 0) s_smin = smin;
  }
  __syncthreads();
  const double smin = s_smin;
  if (!(smin > 0.0) || !isfinite(1.0 / smin)) {
    // sigma_min(A_p) = 0: p is left alone (rank stays P)
    if (t == 0) *d.flag = 1;
    return;
  }
  const double sigma = 1.0 / smin;

  // ---- C = [A_np^T | sigma A_pp^T A_pn]
  for (int q = 0; q < d.nrow; ++q) {
    const T* blk = pool + nb[q].blk;
    const int w = s_w[q], ld = nb[q].ld, o = s_off[q];
    for (int e = t; e < w * P; e += NT) {
      const int b = e / P, a = e - b * P;
      Cw[(int64_t)a * M + o + b] = (double)blk[(int64_t)b * ld + a];
    }
  }
  for (int e = t; e < P * mc; e += NT) {
    const int c = e / P, a = e - c * P;
    const double* ba = B + (int64_t)a * P;
    const double* nc = N + (int64_t)c * P;
    double s0 = 0.0, s1 = 0.0;
    int q = 0;
    for (; q + 1 < P; q += 2) {
      s0 += ba[q] * nc[q];
      s1 += ba[q + 1] * nc[q + 1];
    }
    if (q < P) s0 += ba[q] * nc[q];
    Cw[(int64_t)a * M + mr + c] = sigma * (s0 + s1);
  }
  for (int j = t; j < m; j += NT) perm[j] = j;
  __syncthreads();

  // ---- partial CPQR with exact norms and the ratio rule
  const int kmax = P < m ? P : m;
  int r = 0;
  double R11 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    double bv = -1.0;
    int bi = INT_MAX;
    for (int j = k + t; j < m; j += NT) {
      double s0 = 0.0, s1 = 0.0;
      int i = k;
      for (; i + 1 < P; i += 2) {
        const double v0 = Cw[(int64_t)i * M + j], v1 = Cw[(int64_t)(i + 1) * M + j];
        s0 += v0 * v0;
        s1 += v1 * v1;
      }
      if (i < P) {
        const double v0 = Cw[(int64_t)i * M + j];
        s0 += v0 * v0;
      }
      const double s = s0 + s1;
      if (s > bv) {
        bv = s;
        bi = j;
      }
    }
    u_wg_argmax<NT>(bv, bi, sv, si);
    const double rkk = sqrt(bv);
    if (k == 0) {
      R11 = rkk;
      if (R11 == 0.0) break;
    }
    if (d.eps > 0.0 && rkk < d.eps * R11) break;
    if (bi != k) {
      for (int i = t; i < P; i += NT) {
        const double a = Cw[(int64_t)i * M + k];
        Cw[(int64_t)i * M + k] = Cw[(int64_t)i * M + bi];
        Cw[(int64_t)i * M + bi] = a;
      }
      if (t == 0) {
        const int a = perm[k];
        perm[k] = perm[bi];
        perm[bi] = a;
      }
      __syncthreads();
    }
    double* ck = Cw + (int64_t)k * M + k;
    const double tau = u_larfg<NT>(ck, P - k, M, red);
    if (t == 0) tq[k] = tau;
    for (int u = t; u < P - k; u += NT) vbuf[u] = u == 0 ? 1.0 : ck[(int64_t)u * M];
    __syncthreads();
    if (tau != 0.0)
      for (int j = k + 1 + t; j < m; j += NT) {
        double s0 = 0.0, s1 = 0.0;
        int u = 0;
        for (; u + 1 < P - k; u += 2) {
          s0 += vbuf[u] * Cw[(int64_t)(k + u) * M + j];
          s1 += vbuf[u + 1] * Cw[(int64_t)(k + u + 1) * M + j];
        }
        if (u < P - k) s0 += vbuf[u] * Cw[(int64_t)(k + u) * M + j];
        const double s = (s0 + s1) * tau;
#pragma unroll 4
        for (int q = 0; q < P - k; ++q) Cw[(int64_t)(k + q) * M + j] -= vbuf[q] * s;
      }
    __syncthreads();
    r = k + 1;
  }
  if (r == P) {
    // nothing dropped: p is left alone
    if (t == 0) *d.flag = 1;
    return;
  }
  const int f = P - r;

  // ---- Q's reflectors (unit diagonal), inverse permutation, A_ip Q
  for (int e = t; e < P * r; e += NT) {
    const int c = e / P, i = e - c * P;
    Vq[e] = i < c ? 0.0 : (i == c ? 1.0 : Cw[(int64_t)i * M + c]);
  }
  for (int j = t; j < m; j += NT) iperm[perm[j]] = j;
  __syncthreads();
  for (int q = 0; q < d.nrow; ++q) {
    T* blk = pool + nb[q].blk;
    const int w = s_w[q], ld = nb[q].ld, o = s_off[q];
    for (int e = t; e < w * r; e += NT) {
      const int b = e / r, c = e - b * r;
      const int pos = iperm[o + b];
      blk[(int64_t)b * ld + c] = (T)(c > pos ? 0.0 : Cw[(int64_t)c * M + pos]);
    }
  }

  // ---- A_pp Q = A_pp H_0 H_1 ... H_{r-1}
  for (int u = 0; u < r; ++u) {
    for (int i = t; i < P - u; i += NT) vbuf[i] = Vq[(u + i) + (int64_t)u * P];
    __syncthreads();
    u_right<NT>(vbuf, P - u, tq[u], B + (int64_t)u * P, P, P);
  }

  // ---- Householder QR of the f columns; H^T on the c columns and on A_pn
  for (int u = 0; u < f; ++u) {
    double* bu = B + u + (int64_t)(r + u) * P;
    const double th = u_larfg<NT>(bu, P - u, 1, red);
    if (t == 0) tH[u] = th;
    u_left3<NT>(bu, P - u, th, P, bu + P, f - u - 1, B + u, r, N + u, mc);
  }

  // ---- the new blocks of p: the last r rows, stored first
  for (int e = t; e < r * r; e += NT) {
    const int a = e / r, c = e - a * r;
    app[(int64_t)a * P + c] = (T)B[(f + a) + (int64_t)c * P];
  }
  for (int q = d.nrow; q < nn; ++q) {
    T* blk = pool + nb[q].blk;
    const int w = s_w[q], ld = nb[q].ld, o = s_off[q] - mr;
    for (int e = t; e < r * w; e += NT) {
      const int a = e / w, c = e - a * w;
      blk[(int64_t)a * ld + c] = (T)N[(f + a) + (int64_t)(o + c) * P];
    }
  }

  // ---- forward operator Pi H^T
  for (int e = t; e < P * P; e += NT) E[e] = (e % P == e / P) ? 1.0 : 0.0;
  __syncthreads();
  for (int u = 0; u < f; ++u) u_left<NT>(B + u + (int64_t)(r + u) * P, P - u, tH[u], E + u, P, P);
  for (int e = t; e < P * P; e += NT) {
    const int c = e / P, a = e - c * P;
    const int src = a < r ? f + a : a - r;
    d.mf[e] = (T)E[src + (int64_t)c * P];
  }
  __syncthreads();

  // ---- backward operator Q T
  for (int c = t; c < P; c += NT) {
    double* col = E + (int64_t)c * P;
    for (int i = 0; i < r; ++i) col[i] = i == c ? 1.0 : 0.0;
    for (int b = 0; b < f; ++b) col[r + b] = c < r ? -B[b + (int64_t)c * P] : (b == c - r ? 1.0 : 0.0);
    for (int b = f - 1; b >= 0; --b) {
      double s = col[r + b];
      for (int b2 = b + 1; b2 < f; ++b2) s -= B[b + (int64_t)(r + b2) * P] * col[r + b2];
      col[r + b] = s / B[b + (int64_t)(r + b) * P];
    }
  }
  __syncthreads();
  for (int u = r - 1; u >= 0; --u) u_left<NT>(Vq + u + (int64_t)u * P, P - u, tq[u], E + u, P, P);
  for (int e = t; e < P * P; e += NT) d.mb[e] = (T)E[e];
  if (t == 0) d.rank[d.cluster] = r;
}

// x_p <- M x_p for interfaces of any size up to kSpuMaxP, one workgroup per
// interface: x_p staged in LDS, a thread per row (column-major M, coalesced).
template <typename T>
__global__ void __launch_bounds__(kNTSmall) k_ap_iface_dense_big(const ApIface<T>* __restrict__ ds, int backward,
                                                           double* x, int64_t ldx, int nrhs) {
  __shared__ double xs[kSpuMaxP];
  const ApIface<T> d = ds[blockIdx.x];
  const int P = d.P;
  if (P == 0 || *d.flag != 0) return;
  x += d.xoff;
  const T* Mx = backward ? d.mb : d.mf;
  for (int c = 0; c < nrhs; ++c) {
    for (int i = threadIdx.x; i < P; i += kNTSmall) xs[i] = x[d.slots[i] + (int64_t)c * ldx];
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += kNTSmall) {
      double acc = 0.0;
      for (int j = 0; j < P; ++j) acc += (double)Mx[i + (int64_t)j * P] * xs[j];
      x[d.slots[i] + (int64_t)c * ldx] = acc;
    }
    __syncthreads();
  }
}

void spu_check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string("launch of ") + what + " failed: " + hipGetErrorString(e));
}

}  // namespace

int64_t sparsify_unscaled_ws(int P, int mr_max, int mc_max) {
  const int64_t M = (int64_t)mr_max + mc_max;
  return ((int64_t)P + mr_max) * P + (int64_t)P * M + 3 * (int64_t)P * P + (int64_t)P * mc_max + 4 * (int64_t)P +
         M + 1;
}

template <typename T>
void launch_sparsify_unscaled(const SpuDesc<T>* d, const SpNbr* nb, int64_t n, int max_p, hipStream_t s) {
  if (n <= 0) return;
  count_launch("k_sparsify_unscaled");
  // the launch lasts as long as its slowest interface's chain of reflector
  // steps: 1024 threads shorten every step, and two such workgroups fit a
  // CU, so they pay off until the interfaces outnumber two per CU
  if (max_p <= 64 && n > 512)
    hipLaunchKernelGGL((k_sparsify_unscaled<T, kNTSmall>), dim3((unsigned)n), dim3(kNTSmall), 0, s, d, nb);
  else
    hipLaunchKernelGGL((k_sparsify_unscaled<T, kNTWide>), dim3((unsigned)n), dim3(kNTWide), 0, s, d, nb);
  spu_check_launch("k_sparsify_unscaled");
}

template <typename T>
void launch_iface_dense_big(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                            hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return;
  count_launch("k_ap_iface_dense_big");
  hipLaunchKernelGGL(k_ap_iface_dense_big<T>, dim3((unsigned)n), dim3(kNTSmall), 0, s, d, backward ? 1 : 0, x, ldx,
                     nrhs);
  spu_check_launch("k_ap_iface_dense_big");
}

template void launch_sparsify_unscaled<float>(const SpuDesc<float>*, const SpNbr*, int64_t, int, hipStream_t);
template void launch_sparsify_unscaled<double>(const SpuDesc<double>*, const SpNbr*, int64_t, int, hipStream_t);
template void launch_iface_dense_big<float>(const ApIface<float>*, int64_t, bool, double*, int64_t, int, hipStream_t);
template void launch_iface_dense_big<double>(const ApIface<double>*, int64_t, bool, double*, int64_t, int,
                                             hipStream_t);

}  // namespace spaqr
