// Right-preconditioned flexible GMRES in FP64 on the device (Section 4: GMRES
// with the spaQR factorization as preconditioner, stopping on the relative
// residual).  Several right-hand sides advance together; each keeps its own
// Hessenberg matrix, Givens rotations and stopping point.  Orthogonalization
// is classical Gram-Schmidt applied twice (CGS2): two GEMV-like passes per
// step, which map to wide, barrier-free kernels, instead of j dependent
// passes of modified Gram-Schmidt.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "engine.hpp"
#include "profile.hpp"

namespace spaqr {

namespace {

constexpr int ROWS_PER_BLOCK = 4096;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// y[:, c] = A x[:, c] for CSR A.
__global__ void k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ va, int64_t n, const double* __restrict__ x, int64_t ldx,
                       double* __restrict__ y, int64_t ldy) {
  const int c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t t = rp[r]; t < rp[r + 1]; ++t) s += va[t] * x[ci[t] + c * ldx];
    y[r + c * ldy] = s;
  }
}

// y[:, j] = A_j x[:, j] for column j's own CSR matrix (batched problems).
__global__ void k_spmv_cols(const SpmvCol* __restrict__ sc, const double* __restrict__ x, int64_t ldx,
                            double* __restrict__ y, int64_t ldy) {
  const int j = blockIdx.y;
  const SpmvCol a = sc[j];
  const double* xj = x + (int64_t)j * ldx;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t t = a.rowptr[r]; t < a.rowptr[r + 1]; ++t) s += a.val[t] * xj[a.col[t]];
    y[r + (int64_t)j * ldy] = s;
  }
}

// partial[(c * nblk + blk) * J + j] = sum over the block's rows of
// X[i + j*sj + c*sc] * w[i + c*ldw]; one wavefront per j, no barriers.
__global__ void k_dots(const double* __restrict__ X, int64_t sj, int64_t sc, int J, const double* __restrict__ w,
                       int64_t ldw, int64_t n, double* __restrict__ partial) {
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t r0 = (int64_t)blk * ROWS_PER_BLOCK;
  const int64_t r1 = min(n, r0 + ROWS_PER_BLOCK);
  const double* wc = w + c * ldw;
  for (int j = wv; j < J; j += nw) {
    const double* xj = X + j * sj + c * sc;
    double s = 0.0;
    for (int64_t r = r0 + lane; r < r1; r += 64) s += xj[r] * wc[r];
    s = wsum(s);
    if (lane == 0) partial[((int64_t)c * nblk + blk) * J + j] = s;
  }
}

__global__ void k_reduce(const double* __restrict__ partial, int nblk, int J, int nrhs, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= J * nrhs) return;
  const int c = q / J, j = q - c * J;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[((int64_t)c * nblk + b) * J + j];
  out[q] = s;
}

// w[:, c] += alpha * sum_j X[:, j, c] * h[c*J + j]
__global__ void k_gemv_acc(const double* __restrict__ X, int64_t sj, int64_t sc, int J,
                           const double* __restrict__ h, double alpha, double* __restrict__ w, int64_t ldw,
                           int64_t n) {
  const int c = blockIdx.y;
  const double* hc = h + (int64_t)c * J;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int j = 0; j < J; ++j) s += X[r + j * sj + c * sc] * hc[j];
    w[r + c * ldw] += alpha * s;
  }
}

// dst[:, c] = src[:, c] / s[c] (0 if s[c] == 0)
__global__ void k_scale_cols(const double* __restrict__ src, int64_t lds, const double* __restrict__ s,
                             double* __restrict__ dst, int64_t ldd, int64_t n, int sqrt_s) {
  const int c = blockIdx.y;
  double d = s[c];
  if (sqrt_s) d = sqrt(d);
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    dst[r + c * ldd] = src[r + c * lds] * inv;
}

// y = b - y (column-wise), used for residuals after y = A x
__global__ void k_sub_from(const double* __restrict__ b, int64_t ldb, double* __restrict__ y, int64_t ldy, int64_t n) {
  const int c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    y[r + c * ldy] = b[r + c * ldb] - y[r + c * ldy];
}

__global__ void k_zero_cols(double* x, int64_t ldx, int64_t n) {
  const int c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    x[r + c * ldx] = 0.0;
}

unsigned gx(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

// Solve-scoped device buffer from the stream-ordered pool.
// A pinned host buffer from the recycled pool, returned to it on scope exit
// once the stream has passed every copy that touches it.
struct PinnedHost {
  hipStream_t s;
  PinnedChunk c;
  PinnedHost(size_t bytes, hipStream_t st) : s(st), c(pinned_acquire(bytes)) {}
  ~PinnedHost() {
    (void)hipStreamSynchronize(s);
    pinned_release(c);
  }
  PinnedHost(const PinnedHost&) = delete;
  PinnedHost& operator=(const PinnedHost&) = delete;
};

struct Dev {
  hipStream_t s;
  double* p = nullptr;
  explicit Dev(hipStream_t st) : s(st) {}
  void ensure(size_t n) { p = static_cast<double*>(dev_alloc(std::max<size_t>(1, n) * sizeof(double), s)); }
  void release() {
    dev_free(p, s);
    p = nullptr;
  }
  ~Dev() { release(); }
};

}  // namespace

void launch_spmv(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n, const double* x,
                 int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(gx(n), nrhs), dim3(256), 0, s, rowptr, col, val, n, x, ldx, y, ldy);
}

void launch_spmv_cols(const SpmvCol* sc, int ncols, int64_t max_n, const double* x, int64_t ldx, double* y,
                      int64_t ldy, hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_spmv_cols, dim3(gx(max_n), (unsigned)ncols), dim3(256), 0, s, sc, x, ldx, y, ldy);
}

// h[c*J + j] = X[:, j, c] . w[:, c]
static void dots(const double* X, int64_t sj, int64_t sc, int J, const double* w, int64_t ldw, int64_t n,
                 int nrhs, double* partial, double* out, hipStream_t s) {
  const int nblk = (int)((n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
  hipLaunchKernelGGL(k_dots, dim3(nblk, nrhs), dim3(256), 0, s, X, sj, sc, J, w, ldw, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3((J * nrhs + 255) / 256), dim3(256), 0, s, partial, nblk, J, nrhs, out);
}

int fgmres_solve(KrylovOp& e, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, const double* tol,
                 int restart, int maxit_in, spaqr_solve_info* info, std::vector<double>* history) {
  const double t0 = now_ms();
  hipStream_t s = e.stream();
  const int64_t N = e.n();
  const int m = std::max(1, restart);
  const int maxit = std::max(1, maxit_in);
  const int nblk = (int)((N + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
  Dev V(s), Z(s), W(s), part(s), hd(s);
  HostScope hs_alloc("host_solve_alloc");
  V.ensure((size_t)N * (m + 1) * nrhs);
  // (rows of a column beyond its problem's size, with batched problems, are
  // written by nothing but x += Z y and read by nothing: W and V stay zero there)
  Z.ensure((size_t)N * m * nrhs);
  W.ensure((size_t)N * nrhs);
  part.ensure((size_t)nblk * (m + 2) * nrhs);
  hd.ensure((size_t)(3 * (m + 2)) * nrhs);
  const int64_t sjV = N, scV = N * (m + 1), sjZ = N, scZ = N * m;
  // Step j leaves its projections (two CGS passes, (j + 1) per column each)
  // and the new norms side by side at the start of hd, so one copy brings
  // them to the pinned mirror; y goes up from a pinned region of its own.
  PinnedHost pin((size_t)(3 * m + 3) * nrhs * sizeof(double), s);
  hs_alloc.stop();
  double* hm = reinterpret_cast<double*>(pin.c.p);
  double* ym = hm + (size_t)(2 * m + 3) * nrhs;
  std::vector<double> bnorm(nrhs), rel(nrhs, 1.0);
  std::vector<int> its(nrhs, 0), done(nrhs, 0);
  auto D2H = [&](const double* src, size_t cnt) {
    SPAQR_HIP(hipMemcpyAsync(hm, src, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  };
  // ||b||
  double* hn = hd.p;
  dots(b, 0, ldb, 1, b, ldb, N, nrhs, part.p, hn, s);
  D2H(hn, nrhs);
  SPAQR_HIP(hipStreamSynchronize(s));
  for (int c = 0; c < nrhs; ++c) bnorm[c] = std::sqrt(hm[c]);
  hipLaunchKernelGGL(k_zero_cols, dim3(gx(N), nrhs), dim3(256), 0, s, x, ldx, N);
  // r = b (x0 = 0)
  SPAQR_HIP(hipMemcpy2DAsync(W.p, N * sizeof(double), b, ldb * sizeof(double), N * sizeof(double), nrhs,
                             hipMemcpyDeviceToDevice, s));
  int total = 0;
  std::vector<double> H((size_t)(m + 1) * m * nrhs), cs((size_t)m * nrhs), sn((size_t)m * nrhs),
      g((size_t)(m + 1) * nrhs);
  std::vector<int> jend(nrhs, 0), active(nrhs, 0);
  for (;;) {
    // beta = ||r||
    dots(W.p, 0, N, 1, W.p, N, N, nrhs, part.p, hn, s);
    D2H(hn, nrhs);
    SPAQR_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int c = 0; c < nrhs; ++c) {
      const double beta = std::sqrt(hm[c]);
      rel[c] = bnorm[c] > 0 ? beta / bnorm[c] : 0.0;
      done[c] = rel[c] <= tol[c] || bnorm[c] == 0.0;
      active[c] = !done[c] && its[c] < maxit;
      any = any || active[c];
      std::fill(g.begin() + (size_t)c * (m + 1), g.begin() + (size_t)(c + 1) * (m + 1), 0.0);
      g[(size_t)c * (m + 1)] = beta;
      jend[c] = 0;
    }
    if (!any) break;
    // V_0 = r / beta
    hipLaunchKernelGGL(k_scale_cols, dim3(gx(N), nrhs), dim3(256), 0, s, W.p, N, hn, V.p, scV, N, 1);
    int j = 0;
    for (; j < m; ++j) {
      HostScope hs_launch("host_solve_launch");
      double* Vj = V.p + (size_t)j * sjV;
      double* Zj = Z.p + (size_t)j * sjZ;
      double* h1 = hd.p;
      double* h2 = hd.p + (size_t)(j + 1) * nrhs;
      double* hj = hd.p + (size_t)2 * (j + 1) * nrhs;
      e.apply_dev(Vj, scV, Zj, scZ, nrhs);
      e.spmv_dev(Zj, scZ, W.p, N, nrhs);
      // CGS2
      dots(V.p, sjV, scV, j + 1, W.p, N, N, nrhs, part.p, h1, s);
      hipLaunchKernelGGL(k_gemv_acc, dim3(gx(N), nrhs), dim3(256), 0, s, V.p, sjV, scV, j + 1, h1, -1.0, W.p, N, N);
      dots(V.p, sjV, scV, j + 1, W.p, N, N, nrhs, part.p, h2, s);
      hipLaunchKernelGGL(k_gemv_acc, dim3(gx(N), nrhs), dim3(256), 0, s, V.p, sjV, scV, j + 1, h2, -1.0, W.p, N, N);
      dots(W.p, 0, N, 1, W.p, N, N, nrhs, part.p, hj, s);
      hipLaunchKernelGGL(k_scale_cols, dim3(gx(N), nrhs), dim3(256), 0, s, W.p, N, hj, V.p + (size_t)(j + 1) * sjV,
                         scV, N, 1);
      D2H(hd.p, (size_t)(2 * (j + 1) + 1) * nrhs);
      hs_launch.stop();
      {
        HostScope hs_sync("host_solve_sync");
        SPAQR_HIP(hipStreamSynchronize(s));
      }
      const double* hh1 = hm;
      const double* hh2 = hm + (size_t)(j + 1) * nrhs;
      const double* hhn = hm + (size_t)2 * (j + 1) * nrhs;
      bool still = false;
      for (int c = 0; c < nrhs; ++c) {
        if (!active[c]) continue;
        double* Hc = H.data() + (size_t)c * (m + 1) * m;  // column-major (m+1) x m
        double* col = Hc + (size_t)j * (m + 1);
        for (int i = 0; i <= j; ++i) col[i] = hh1[(size_t)c * (j + 1) + i] + hh2[(size_t)c * (j + 1) + i];
        col[j + 1] = std::sqrt(hhn[c]);
        double* csc = cs.data() + (size_t)c * m;
        double* snc = sn.data() + (size_t)c * m;
        double* gc = g.data() + (size_t)c * (m + 1);
        for (int i = 0; i < j; ++i) {
          const double t = csc[i] * col[i] + snc[i] * col[i + 1];
          col[i + 1] = -snc[i] * col[i] + csc[i] * col[i + 1];
          col[i] = t;
        }
        const double den = std::hypot(col[j], col[j + 1]);
        if (den == 0.0) {
          csc[j] = 1.0;
          snc[j] = 0.0;
        } else {
          csc[j] = col[j] / den;
          snc[j] = col[j + 1] / den;
        }
        col[j] = csc[j] * col[j] + snc[j] * col[j + 1];
        col[j + 1] = 0.0;
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        its[c]++;
        jend[c] = j + 1;
        const double est = std::fabs(gc[j + 1]) / bnorm[c];
        if (history && c == 0) history->push_back(est);
        if (est <= tol[c] || its[c] >= maxit || col[j] == 0.0) active[c] = 0;
        still = still || active[c];
      }
      total = *std::max_element(its.begin(), its.end());
      if (!still) break;
    }
    // x += Z y per column
    const int J = std::min(m, std::max(1, *std::max_element(jend.begin(), jend.end())));
    double* y = ym;
    std::fill(y, y + (size_t)J * nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) {
      const double* Hc = H.data() + (size_t)c * (m + 1) * m;
      const double* gc = g.data() + (size_t)c * (m + 1);
      for (int i = jend[c] - 1; i >= 0; --i) {
        double sacc = gc[i];
        for (int q = i + 1; q < jend[c]; ++q) sacc -= Hc[i + (size_t)q * (m + 1)] * y[(size_t)c * J + q];
        y[(size_t)c * J + i] = Hc[i + (size_t)i * (m + 1)] != 0.0 ? sacc / Hc[i + (size_t)i * (m + 1)] : 0.0;
      }
    }
    // (the pinned y is rewritten only after the next synchronization)
    SPAQR_HIP(hipMemcpyAsync(hd.p, y, (size_t)J * nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gemv_acc, dim3(gx(N), nrhs), dim3(256), 0, s, Z.p, sjZ, scZ, J, hd.p, 1.0, x, ldx, N);
    // r = b - A x
    e.spmv_dev(x, ldx, W.p, N, nrhs);
    hipLaunchKernelGGL(k_sub_from, dim3(gx(N), nrhs), dim3(256), 0, s, b, ldb, W.p, N, N);
    bool more = false;
    for (int c = 0; c < nrhs; ++c) more = more || its[c] < maxit;
    if (!more) {
      dots(W.p, 0, N, 1, W.p, N, N, nrhs, part.p, hn, s);
      D2H(hn, nrhs);
      SPAQR_HIP(hipStreamSynchronize(s));
      for (int c = 0; c < nrhs; ++c) {
        rel[c] = bnorm[c] > 0 ? std::sqrt(hm[c]) / bnorm[c] : 0.0;
        done[c] = rel[c] <= tol[c] || bnorm[c] == 0.0;
      }
      break;
    }
  }
  SPAQR_HIP(hipGetLastError());
  if (history) history->push_back(rel[0]);
  const double dt = (now_ms() - t0) / 1000.0;
  int status = SPAQR_OK;
  for (int c = 0; c < nrhs; ++c) {
    if (!done[c]) status = SPAQR_ENOCONV;
    if (info) {
      info[c].iterations = its[c];
      info[c].converged = done[c];
      info[c].relres = rel[c];
      info[c].seconds = dt;
    }
  }
  (void)total;
  return status;
}

int fgmres_solve_batch(const std::vector<EngineBase*>& es, const std::vector<int>& nrhs,
                       const std::vector<const double*>& b, const std::vector<double*>& x,
                       const std::vector<double>& tol, spaqr_solve_info* info, std::vector<int>* status) {
  const size_t np = es.size();
  SPAQR_REQUIRE(np > 0 && nrhs.size() == np && b.size() == np && x.size() == np && tol.size() == np, SPAQR_EINVAL,
                "batched solve: argument lists differ in length");
  std::unique_ptr<KrylovOp> op;
  {
    HostScope hs("host_solve_setup");
    op = make_batch_op(es, nrhs);
  }
  HostScope hs_all("host_solve_krylov");
  hipStream_t s = op->stream();
  const int64_t N = op->n();
  int C = 0, restart = 1, maxit = 1;
  std::vector<int> c0(np);
  std::vector<double> tc;
  for (size_t i = 0; i < np; ++i) {
    c0[i] = C;
    C += nrhs[i];
    restart = std::max(restart, es[i]->opt_restart());
    maxit = std::max(maxit, es[i]->opt_maxit());
    tc.insert(tc.end(), (size_t)nrhs[i], tol[i]);
  }
  Dev B(s), X(s);
  B.ensure((size_t)N * C);
  X.ensure((size_t)N * C);
  // columns padded to the largest n with zeros
  SPAQR_HIP(hipMemsetAsync(B.p, 0, (size_t)N * C * sizeof(double), s));
  for (size_t i = 0; i < np; ++i) {
    const int64_t n = es[i]->n();
    SPAQR_HIP(hipMemcpy2DAsync(B.p + (size_t)c0[i] * N, N * sizeof(double), b[i], n * sizeof(double),
                               n * sizeof(double), nrhs[i], hipMemcpyDeviceToDevice, s));
  }
  std::vector<spaqr_solve_info> inf((size_t)C);
  fgmres_solve(*op, B.p, N, X.p, N, C, tc.data(), restart, maxit, inf.data());
  int st = SPAQR_OK;
  if (status) status->assign(np, SPAQR_OK);
  for (size_t i = 0; i < np; ++i) {
    const int64_t n = es[i]->n();
    SPAQR_HIP(hipMemcpy2DAsync(x[i], n * sizeof(double), X.p + (size_t)c0[i] * N, N * sizeof(double),
                               n * sizeof(double), nrhs[i], hipMemcpyDeviceToDevice, s));
    for (int r = 0; r < nrhs[i]; ++r)
      if (!inf[(size_t)c0[i] + r].converged) {
        st = SPAQR_ENOCONV;
        if (status) (*status)[i] = SPAQR_ENOCONV;
      }
  }
  SPAQR_HIP(hipStreamSynchronize(s));
  X.release();
  B.release();
  if (info) std::copy(inf.begin(), inf.end(), info);
  return st;
}

}  // namespace spaqr
