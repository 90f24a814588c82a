// Numeric spaQR engine: device memory, the stage-by-stage factorization
// driver, the preconditioner apply and FGMRES.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mem.hpp"
#include "symbolic.hpp"

namespace spaqr {

#define SPAQR_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::spaqr::Error(SPAQR_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over stream-ordered device chunks.
class DevArena {
 public:
  explicit DevArena(size_t chunk = size_t(32) << 20) : chunk_(chunk) {}
  ~DevArena();
  void* alloc(size_t bytes, hipStream_t s);
  template <typename X>
  X* alloc_n(size_t n, hipStream_t s) { return static_cast<X*>(alloc(n * sizeof(X), s)); }
  void reset() { cur_ = 0; off_ = 0; used_ = 0; }
  void release(hipStream_t s);
  size_t reserved() const;
  size_t used() const { return used_; }  // bytes handed out since the last reset

 private:
  struct Chunk { char* p; size_t size; };
  std::vector<Chunk> chunks_;
  size_t chunk_, cur_ = 0, off_ = 0, used_ = 0;
  hipStream_t stream_ = nullptr;  // stream of the allocations (frees are ordered on it)
};

// Pinned host staging for uploads; reset only once the stream has passed
// every copy issued from it.
class Stager {
 public:
  ~Stager();
  template <typename X>
  X* upload(DevArena& arena, const std::vector<X>& v, hipStream_t s) {
    if (v.empty()) return nullptr;
    return static_cast<X*>(upload_bytes(arena, v.data(), v.size() * sizeof(X), s));
  }
  void* upload_bytes(DevArena& arena, const void* src, size_t bytes, hipStream_t s);
  // two-step upload: stage() hands out a pinned host region and its device
  // destination, the caller fills the host side, send() issues the copy
  struct Region {
    void* host;
    void* dev;
    size_t bytes;
  };
  Region stage(DevArena& arena, size_t bytes, hipStream_t s);
  void send(const Region& r, hipStream_t s);
  // like upload(), but the copy is held back and merged with the next
  // held-back upload when both are contiguous on the host and the device
  // (consecutive uploads into one arena chunk): flush() must be called
  // before anything on the stream reads the data
  template <typename X>
  X* upload_held(DevArena& arena, const std::vector<X>& v, hipStream_t s) {
    if (v.empty()) return nullptr;
    return static_cast<X*>(upload_held_bytes(arena, v.data(), v.size() * sizeof(X), s));
  }
  void* upload_held_bytes(DevArena& arena, const void* src, size_t bytes, hipStream_t s);
  void flush(hipStream_t s);
  void reset() {
    cur_ = 0;
    off_ = 0;
    held_ = Region{nullptr, nullptr, 0};
  }

 private:
  std::vector<PinnedChunk> chunks_;
  size_t cur_ = 0, off_ = 0;
  Region held_{nullptr, nullptr, 0};
};

template <typename T>
struct StageApply {
  ApFront<T>* fronts = nullptr;          // colour order
  std::vector<int64_t> colour_ptr;       // boundaries of colours in fronts
  std::vector<int> colour_max_m;         // LDS rows of the forward launch per colour
  int max_bwd_rows = 0;                  // max n + k
  int max_n = 0, max_k = 0;              // largest front and ancestor-column widths
  int jb = 1;                            // QR panel width of the stage's fronts
  int64_t nifaces_small = 0;             // interfaces with dense operators come first
  int dense_max = 64;                    // largest interface given dense operators
  int dense_max_p = 0;                   // largest interface that has them
  int64_t nfronts = 0;
  ApIface<T>* ifaces = nullptr;
  int64_t nifaces = 0;
  int max_p = 0;
  // algorithmic work of each apply launch: factor + index bytes (read once per
  // launch) and per-right-hand-side vector bytes and flops
  std::vector<double> fwd_fac_bytes, fwd_vec_bytes, fwd_flops;  // per colour
  double bwd_fac_bytes = 0, bwd_vec_bytes = 0, bwd_flops = 0;
  double if_fwd_fac_bytes = 0, if_bwd_fac_bytes = 0, if_vec_bytes = 0, if_fwd_flops = 0, if_bwd_flops = 0;
  // host copies of the descriptors (fronts in colour order, interfaces with
  // the dense-operator ones first), for applies batched across problems
  std::vector<ApFront<T>> h_fronts;
  std::vector<ApIface<T>> h_ifaces;
};

struct Stats {
  spaqr_stats_t s{};
  std::vector<std::vector<int32_t>> stage_sizes;  // index k: sizes after stage k
  std::vector<spaqr_stage_stats_t> stage;         // index k: per-stage statistics
  std::vector<std::vector<int32_t>> ifaces;       // index k: (cluster, |p|, m_p, r_p) per interface
  std::vector<double> history;                    // last solve: residual estimates, then the true residual
};

// HIP events around the phases of one batched stage: start, after the fronts,
// after the scaling, after the sparsification, after the merge.  Shared by the
// factorizations advanced together in that stage.
struct PhaseEvents {
  hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  PhaseEvents();
  ~PhaseEvents();
  PhaseEvents(const PhaseEvents&) = delete;
  PhaseEvents& operator=(const PhaseEvents&) = delete;
  void record(int i, hipStream_t s);
  double ms(int i) const;  // elapsed between e[i] and e[i + 1] (the events must be complete), 0 if unrecorded

 private:
  unsigned done_ = 0;  // bit i: e[i] recorded
};

// What FGMRES needs of a system: n rows per column, the preconditioner and
// the matrix applied to ncols columns at once (device pointers, column-major).
class KrylovOp {
 public:
  virtual ~KrylovOp() = default;
  // x = M^{-1} b
  virtual void apply_dev(const double* b, int64_t ldb, double* x, int64_t ldx, int ncols) = 0;
  // y = A x
  virtual void spmv_dev(const double* x, int64_t ldx, double* y, int64_t ldy, int ncols) = 0;
  virtual hipStream_t stream() const = 0;
  virtual int64_t n() const = 0;
};

class EngineBase : public KrylovOp {
 public:
  // x = M^{-1} b with the caller's workspace ws (n * nrhs doubles) for the
  // permuted vectors: enqueued on stream(), allocates nothing
  virtual void apply_ws(const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, double* ws) = 0;
  virtual const Stats& stats() const = 0;
  virtual int opt_restart() const = 0;
  virtual int opt_maxit() const = 0;
  virtual int stages_left() const = 0;  // 0 once the factorization is complete (or failed)
  virtual int precision() const = 0;    // 32 or 64
  virtual int error() const = 0;        // SPAQR_OK, or the status of a failed factorization
  virtual void set_history(std::vector<double> h) = 0;  // residual history of the last solve
  virtual const char* error_message() const = 0;
};

// A: host CSR (the pattern is always read; values only when Ad is null).
// Ad: optional device copies of the same CSR, used instead of uploading.
std::unique_ptr<EngineBase> make_engine(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S,
                                        const spaqr_opts& o, hipStream_t stream);
// The same, with the stages left to factor_stage_batch (A is read during the
// call only).
std::unique_ptr<EngineBase> make_engine_deferred(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S,
                                                 const spaqr_opts& o, hipStream_t stream);
// Advances every factorization in es by one stage, concatenating their launch
// lists phase by phase (cross-request batching); es share stream s.
struct BatchDriver;
BatchDriver* batch_driver_new();
void batch_driver_free(BatchDriver* d);
void factor_stage_batch(BatchDriver& drv, const std::vector<EngineBase*>& es, hipStream_t s);

// Several factorizations as one block-diagonal operator for FGMRES: problem
// i owns nrhs[i] consecutive columns, problems in the order of es; the
// factorizations must share one stream.  n() is the largest n; rows of a
// column beyond its problem's n are neither read nor written.  Every apply
// runs one launch per phase for all problems (cross-request batching).
std::unique_ptr<KrylovOp> make_batch_op(const std::vector<EngineBase*>& es, const std::vector<int>& nrhs);

// FGMRES on the device (gmres.hip); tol holds one tolerance per column.
int fgmres_solve(KrylovOp& op, const double* b, int64_t ldb, double* x, int64_t ldx, int ncols,
                 const double* tol, int restart, int maxit, spaqr_solve_info* info,
                 std::vector<double>* history = nullptr);
// FGMRES for several factored problems at once (make_batch_op): problem i
// solves nrhs[i] columns b[i] -> x[i] (device, column-major, ld = its n) to
// tol[i].  info receives one entry per column in problem order; status (may
// be null) one per problem (OK or ENOCONV).  Returns ENOCONV if any column
// did not converge.
int fgmres_solve_batch(const std::vector<EngineBase*>& es, const std::vector<int>& nrhs,
                       const std::vector<const double*>& b, const std::vector<double*>& x,
                       const std::vector<double>& tol, spaqr_solve_info* info, std::vector<int>* status);

double now_ms();

}  // namespace spaqr

struct spaqr_handle {
  std::unique_ptr<spaqr::EngineBase> e;
  std::unique_ptr<spaqr::Symbolic> owned_sym;
};
