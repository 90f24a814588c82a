// Stage-by-stage numeric factorization (Algorithm 2) and preconditioner apply.
//
// Memory layout in HBM.  Each stage k has a pool holding every block of the
// stage (pattern at stage start plus the fill of its fronts), row-major with
// the leading dimension equal to the column cluster's size when the stage
// began.  Sparsification shrinks blocks in place (the leading dimension stays);
// current sizes live in a device table that the sparsify kernels read.  After
// a stage the host reads the ranks back once, lays out the next pool with the
// compressed sizes and merges child blocks into it.  Factors (front V/R_ss,
// R_sj, scaling U/R_pp, sparsification Q) are stored column-major for the
// apply and stay resident for the handle's lifetime.  Vectors live in the
// permuted index space ("slots"); a cluster owns a list of slots, sparsification
// keeps its first r slots as the coarse unknowns, and a merge concatenates
// slot lists without moving data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <string>

#include "engine.hpp"
#include "pool.hpp"
#include "profile.hpp"

namespace spaqr {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- DevArena
DevArena::~DevArena() {
  for (auto& c : chunks_) dev_free(c.p, stream_);
}

void* DevArena::alloc(size_t bytes, hipStream_t s) {
  bytes = (bytes + 255) & ~size_t(255);
  if (bytes == 0) bytes = 256;
  used_ += bytes;
  while (cur_ < chunks_.size()) {
    if (off_ + bytes <= chunks_[cur_].size) {
      void* p = chunks_[cur_].p + off_;
      off_ += bytes;
      return p;
    }
    ++cur_;
    off_ = 0;
  }
  const size_t sz = std::max(chunk_, bytes);
  char* p = static_cast<char*>(dev_alloc(sz, s));
  stream_ = s;
  chunks_.push_back({p, sz});
  cur_ = chunks_.size() - 1;
  off_ = bytes;
  return p;
}

void DevArena::release(hipStream_t s) {
  for (auto& c : chunks_) dev_free(c.p, s);
  chunks_.clear();
  reset();
}

size_t DevArena::reserved() const {
  size_t t = 0;
  for (auto& c : chunks_) t += c.size;
  return t;
}

// ---------------------------------------------------------------- Stager
Stager::~Stager() {
  for (auto& c : chunks_) pinned_release(c);
}

Stager::Region Stager::stage(DevArena& arena, size_t bytes, hipStream_t s) {
  void* dst = arena.alloc(bytes, s);
  size_t need = (bytes + 255) & ~size_t(255);
  while (cur_ < chunks_.size() && off_ + need > chunks_[cur_].size) {
    ++cur_;
    off_ = 0;
  }
  if (cur_ >= chunks_.size()) {
    chunks_.push_back(pinned_acquire(need));
    cur_ = chunks_.size() - 1;
    off_ = 0;
  }
  char* h = chunks_[cur_].p + off_;
  off_ += need;
  return {h, dst, bytes};
}

void Stager::send(const Region& r, hipStream_t s) {
  if (r.bytes) SPAQR_HIP(hipMemcpyAsync(r.dev, r.host, r.bytes, hipMemcpyHostToDevice, s));
}

void* Stager::upload_held_bytes(DevArena& arena, const void* src, size_t bytes, hipStream_t s) {
  const Region r = stage(arena, bytes, s);
  std::memcpy(r.host, src, bytes);
  if (held_.bytes) {
    // both sides hand out 256-byte granules, so the held region ends where
    // its padded size ends
    const size_t pad = (held_.bytes + 255) & ~size_t(255);
    if (static_cast<char*>(held_.host) + pad == r.host && static_cast<char*>(held_.dev) + pad == r.dev) {
      held_.bytes = pad + bytes;
      return r.dev;
    }
    flush(s);
  }
  held_ = r;
  return r.dev;
}

void Stager::flush(hipStream_t s) {
  if (held_.bytes) send(held_, s);
  held_ = Region{nullptr, nullptr, 0};
}

void* Stager::upload_bytes(DevArena& arena, const void* src, size_t bytes, hipStream_t s) {
  const Region r = stage(arena, bytes, s);
  std::memcpy(r.host, src, bytes);
  send(r, s);
  return r.dev;
}

void launch_spmv(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n, const double* x,
                 int64_t ldx, double* y, int64_t ldy, int nrhs, hipStream_t s);

PhaseEvents::PhaseEvents() {
  for (auto& ev : e) SPAQR_HIP(hipEventCreate(&ev));
}

PhaseEvents::~PhaseEvents() {
  for (auto& ev : e)
    if (ev) (void)hipEventDestroy(ev);
}

void PhaseEvents::record(int i, hipStream_t s) {
  SPAQR_HIP(hipEventRecord(e[i], s));
  done_ |= 1u << i;
}

double PhaseEvents::ms(int i) const {
  float t = 0.f;
  if (!(done_ >> i & 1u) || !(done_ >> (i + 1) & 1u)) return 0.0;
  return hipEventElapsedTime(&t, e[i], e[i + 1]) == hipSuccess ? (double)t : 0.0;
}

namespace {

struct ZeroOp {
  void* p;
  int64_t bytes;
};

template <typename X>
void append(std::vector<X>& dst, const std::vector<X>& src) {
  dst.insert(dst.end(), src.begin(), src.end());
}

// One stage of one factorization as host-side launch lists.  Every device
// pointer in them is absolute, so the lists of several factorizations (each
// at its own stage) concatenate into one launch per phase.
template <typename T>
struct StagePlan {
  std::vector<ZeroOp> zero;  // runs first
  struct FrontColour {
    // copy tiles in chunks (planned in parallel), launched as one list
    std::vector<std::vector<CopyTile<T>>> gather, scatter;
    std::vector<QRDesc<T>> qr;
    // fronts with many trailing columns or rows: pivot block factored alone,
    // trailing columns updated slice by slice
    std::vector<TrailDesc<T>> trail;
    // the same on the matrix cores: T factors of 64-reflector blocks, then
    // 64-column tiles
    std::vector<WYBlock<T>> wyb;
    std::vector<WYTile<T>> wyt;
    int trail_cw = 0, trail_max_m = 1;
    int max_m = 1;
    double flops = 0.0, bytes = 0.0;
  };
  std::vector<FrontColour> fronts;
  int jbf = 16;
  std::vector<CopyTile<T>> pack;
  // block-diagonal scaling
  std::vector<CopyTile<T>> sgather, spack;
  std::vector<QRDesc<T>> sqr;
  int max_p = 1, jbs = 16;
  std::vector<ScaleFac<T>> fac;
  std::vector<ScaleBlk<T>> sblk;  // fi, fj index fac
  // sparsification, colour by colour; SpDesc::nb indexes nb of its colour
  struct SpColour {
    std::vector<SpDesc<T>> sd;
    std::vector<SpNbr> nb;
  };
  std::vector<SpColour> sp;
  // sparsification without scaling, colour by colour; SpuDesc::nb indexes nb
  struct SpuColour {
    std::vector<SpuDesc<T>> sd;
    std::vector<SpNbr> nb;
  };
  std::vector<SpuColour> spu;
  // interfaces whose dense apply operators are formed after the stage
  std::vector<ApIface<T>> form;
};

template <typename T>
struct MergePlan {
  std::vector<ZeroOp> zero;
  std::vector<std::vector<CopyTile<T>>> tiles;  // in chunks (planned in parallel), launched as one list
};

// A graph of the launches fn(stream) issues, captured on a private stream of
// its own: capture records the launches without running them (and the legacy
// null stream a caller may pass cannot be captured); the graph is then
// launched on the caller's stream.
static hipGraphExec_t capture_graph(const std::function<void(hipStream_t)>& fn) {
  hipStream_t cs = nullptr;
  SPAQR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    try {
      fn(cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      throw;
    }
    e = hipStreamEndCapture(cs, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) throw Error(SPAQR_EDEVICE, std::string("graph capture of the apply failed: ") + hipGetErrorString(e));
  return ex;
}

template <typename T>
class Engine final : public EngineBase {
 public:
  Engine(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S, const spaqr_opts& o, hipStream_t s)
      : S_(S), o_(o), s_(s) {
    mem_setup(s_);
    st_.s.n = S.n;
    st_.s.levels = S.L;
    st_.s.precision = sizeof(T) == 4 ? 32 : 64;
    st_.s.ms_symbolic = S.ms_analysis;
    st_.stage_sizes.assign(S.L + 1, {});
    st_.stage.assign(S.L + 1, spaqr_stage_stats_t{});
    st_.ifaces.assign(S.L + 1, {});
    pev_.assign(S.L + 1, nullptr);
    t0_ = now_ms();
    try {
      begin(A, Ad);
    } catch (...) {
      (void)hipStreamSynchronize(s_);
      throw;
    }
  }
  ~Engine() override {
    drop_graphs();
    dev_free(apply_ws_, s_);
    (void)hipStreamSynchronize(s_);
  }

  void apply_dev(const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs) override;
  void apply_ws(const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, double* ws) override;
  // the two sweeps of the apply on the permuted vectors xh, enqueued on s
  // (the handle's stream unless being captured)
  void sweeps(double* xh, int nrhs, hipStream_t s);
  void sweeps(double* xh, int nrhs) { sweeps(xh, nrhs, s_); }
  void spmv_dev(const double* x, int64_t ldx, double* y, int64_t ldy, int nrhs) override {
    launch_spmv(d_rowptr_, d_col_, d_val_, S_.n, x, ldx, y, ldy, nrhs, s_);
  }
  const Stats& stats() const override { return st_; }
  hipStream_t stream() const override { return s_; }
  int64_t n() const override { return S_.n; }
  int opt_restart() const override { return o_.restart; }
  int opt_maxit() const override { return o_.maxit; }
  int stages_left() const override { return k_; }
  int precision() const override { return sizeof(T) == 4 ? 32 : 64; }
  int error() const override { return err_; }
  const char* error_message() const override { return err_msg_.c_str(); }
  void set_history(std::vector<double> h) override { st_.history = std::move(h); }
  // the phase events of the stage being run (shared by a batch)
  void note_phases(const std::shared_ptr<PhaseEvents>& pe) {
    if (k_ > 0) pev_[k_] = pe;
  }

  // what an apply batched across problems reads
  const std::vector<StageApply<T>>& stage_apply() const { return ap_; }
  int levels() const { return S_.L; }
  const int64_t* perm_dev() const { return d_perm_; }
  const double* colscale_dev() const { return d_dc_; }
  SpmvCol spmv_col() const { return {d_rowptr_, d_col_, d_val_, S_.n}; }

  // stage k_ as launch lists, in three parts that the driver launches in
  // turn: fronts (and the factor packing), scaling, sparsification (each
  // allocates this factorization's buffers for its part)
  void plan_fronts(StagePlan<T>& p);
  void plan_scale(StagePlan<T>& p);
  void plan_sparsify(StagePlan<T>& p);
  void plan_sparsify_unscaled(StagePlan<T>& p);
  // after the launches: the ranks and error flags of the stage, as copies
  // into a batch-wide buffer from offset base (readback_ints() of them);
  // finish() reads them at `host` once the stream has passed the copy
  int readback_ints() const { return (int)S_.st[k_].nclu + 2; }
  void readback_ops(std::vector<IntCopy>& ops, int32_t base) const;
  void readback_to(const int* host) { rb_ = host; }
  // host threads the planning of this factorization may use (null: none)
  void set_host_pool(HostPool* p) { inner_pool_ = p; }
  // after the stream synchronized: sizes and accounting of stage k_, the
  // merge to stage k_ - 1 as launch lists, then k_ <- k_ - 1
  void finish(MergePlan<T>& mp);

 private:
  void begin(const spaqr_csr* A, const spaqr_csr_dev* Ad);
  void complete();
  void begin_stage();

  const Symbolic& S_;
  spaqr_opts o_;
  hipStream_t s_;
  Stats st_;
  double t0_ = 0.0;
  int k_ = 0;  // next stage to run (L .. 1); 0 when the factorization is complete
  int err_ = SPAQR_OK;  // a failed factorization stops with k_ = 0 and this status
  std::string err_msg_;
  DevArena persist_{size_t(64) << 20};
  DevArena work_{size_t(64) << 20};
  DevArena pools_[2] = {DevArena(size_t(64) << 20), DevArena(size_t(64) << 20)};
  Stager stager_[2];
  int stager_cur_ = 0;
  std::vector<std::shared_ptr<PhaseEvents>> pev_;  // index k: events of stage k's phases
  size_t persist_mark_ = 0;                         // factor bytes at the start of the stage
  const int* rb_ = nullptr;  // ranks, zero-diagonal flag, zero-column flag of the stage (host)
  int* d_zcol_ = nullptr;  // set by the device column-norm kernel for a zero column
  int* d_flag_ = nullptr;  // zero R_ss diagonal in a front of the current stage
  int* d_rank_ = nullptr;  // current cluster sizes of the current stage
  HostPool* inner_pool_ = nullptr;  // threads for planning this factorization alone (batch of one)
  // interfaces of the current stage: index by cluster, offsets and buffers
  struct IfaceBufs {
    std::vector<int32_t> fidx;
    std::vector<int64_t> u_off, p_off, t_off;
    T *vru = nullptr, *tauu = nullptr, *tpan = nullptr, *vq = nullptr, *tauq = nullptr;
    int* flags = nullptr;
  } ib_;

  // current stage state
  T* pool_ = nullptr;
  std::vector<int64_t> boff_;       // block offsets (elements) in the pool, by S_.st[k].all index
  std::vector<int32_t> size_;       // current cluster sizes (alloc sizes of the pool)
  std::vector<int64_t> slot_ptr_;   // slot lists of the current clusters
  std::vector<int32_t> slots_;

  // apply data
  std::vector<StageApply<T>> ap_;
  int64_t* d_perm_ = nullptr;
  double* d_dc_ = nullptr;
  int64_t* d_rowptr_ = nullptr;
  int32_t* d_col_ = nullptr;
  double* d_val_ = nullptr;
  double* apply_ws_ = nullptr;
  size_t apply_ws_cap_ = 0;
  // sweeps of apply_dev captured per width nrhs (null: seen once, not yet
  // captured); they read apply_ws_, so they are dropped when it moves
  std::map<int, hipGraphExec_t> graphs_;
  hipGraphExec_t capture_sweeps(double* xh, int nrhs);
  void drop_graphs();
};

template <typename T>
void Engine<T>::begin_stage() {
  stager_cur_ ^= 1;
  stager_[stager_cur_].reset();
  work_.reset();
}

template <typename T>
void Engine<T>::begin(const spaqr_csr* A, const spaqr_csr_dev* Ad) {
  const int L = S_.L;
  const int64_t n = S_.n, nnz = S_.nnz;
  const Ordering& ord = S_.ord;
  ap_.assign(L + 1, StageApply<T>());
  begin_stage();
  Stager& up = stager_[stager_cur_];
  d_perm_ = up.upload(persist_, ord.perm, s_);
  d_zcol_ = persist_.alloc_n<int>(1, s_);
  launch_fill<int>(d_zcol_, 1, 0, s_);
  std::vector<double> dc;
  HostScope hs_csr("host_setup_csr");
  // the analysis's pattern maps in one copy, straight from its pinned buffer
  // when it has one
  const size_t maps_bytes = S_.maps_words() * sizeof(int64_t);
  int64_t* d_maps = nullptr;
  if (S_.maps.pinned()) {
    d_maps = work_.alloc_n<int64_t>(S_.maps_words(), s_);
    SPAQR_HIP(hipMemcpyAsync(d_maps, S_.maps.data(), maps_bytes, hipMemcpyHostToDevice, s_));
  } else {
    d_maps = static_cast<int64_t*>(up.upload_bytes(work_, S_.maps.data(), maps_bytes, s_));
  }
  int64_t* d_cptr = d_maps;
  int64_t* d_cidx = d_cptr + (n + 1);
  int64_t* d_dst = d_cidx + nnz;
  if (Ad) {
    // values already on the device: copy the CSR (device to device) for the
    // SpMV and compute the column scaling there, in a fixed summation order
    d_rowptr_ = persist_.alloc_n<int64_t>(n + 1, s_);
    d_col_ = persist_.alloc_n<int32_t>(std::max<int64_t>(1, nnz), s_);
    d_val_ = persist_.alloc_n<double>(std::max<int64_t>(1, nnz), s_);
    SPAQR_HIP(hipMemcpyAsync(d_rowptr_, Ad->rowptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToDevice, s_));
    SPAQR_HIP(hipMemcpyAsync(d_col_, Ad->col, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s_));
    SPAQR_HIP(hipMemcpyAsync(d_val_, Ad->val, nnz * sizeof(double), hipMemcpyDeviceToDevice, s_));
    d_dc_ = persist_.alloc_n<double>(n, s_);
    launch_colnorm(d_cptr, d_cidx, d_val_, n, d_dc_, d_zcol_, s_);
  } else {
    // Section 2.8: pre-scale columns to unit 2-norm.
    std::vector<double> cn(n, 0.0);
    for (int64_t t = 0; t < nnz; ++t) cn[A->col[t]] += A->val[t] * A->val[t];
    dc.resize(n);
    for (int64_t j = 0; j < n; ++j) {
      SPAQR_REQUIRE(cn[j] > 0.0, SPAQR_EINVAL, "A has a zero column");
      dc[j] = 1.0 / std::sqrt(cn[j]);
    }
    d_dc_ = up.upload(persist_, dc, s_);
    d_rowptr_ = static_cast<int64_t*>(up.upload_bytes(persist_, A->rowptr, (size_t)(n + 1) * sizeof(int64_t), s_));
    d_col_ = nnz ? static_cast<int32_t*>(up.upload_bytes(persist_, A->col, (size_t)nnz * sizeof(int32_t), s_))
                 : persist_.alloc_n<int32_t>(1, s_);
    d_val_ = nnz ? static_cast<double*>(up.upload_bytes(persist_, A->val, (size_t)nnz * sizeof(double), s_))
                 : persist_.alloc_n<double>(1, s_);
  }
  hs_csr.stop();
  HostScope hs_pool("host_setup_pool");
  // stage-L clusters, slots and pool
  const StageClusters& cl = ord.stages[L];
  size_.resize(cl.count());
  slot_ptr_.assign(cl.count() + 1, 0);
  slots_.resize(n);
  for (int64_t c = 0; c < cl.count(); ++c) {
    size_[c] = (int32_t)(cl.end[c] - cl.start[c]);
    slot_ptr_[c + 1] = slot_ptr_[c] + size_[c];
    for (int64_t p = cl.start[c]; p < cl.end[c]; ++p) slots_[p] = (int32_t)p;
  }
  boff_ = S_.pool_off_L;
  pools_[L & 1].reset();
  pool_ = pools_[L & 1].alloc_n<T>(std::max<int64_t>(1, boff_.back()), s_);
  launch_fill<T>(pool_, boff_.back(), T(0), s_);
  {
    launch_scatter_scaled<T>(pool_, d_dst, d_val_, d_col_, d_dc_, nnz, s_);
  }
  k_ = L;
  rb_ = nullptr;
}

template <typename T>
void Engine<T>::complete() {
  SPAQR_HIP(hipStreamSynchronize(s_));
  st_.s.factor_bytes = (int64_t)persist_.used();
  for (int k = 1; k <= S_.L; ++k) {
    if (!pev_[k]) continue;
    spaqr_stage_stats_t& sg = st_.stage[k];
    sg.ms_front = pev_[k]->ms(0);
    sg.ms_scale = pev_[k]->ms(1);
    sg.ms_sparsify = pev_[k]->ms(2);
    sg.ms_merge = pev_[k]->ms(3);
    st_.s.ms_phase[0] += sg.ms_front;
    st_.s.ms_phase[1] += sg.ms_scale;
    st_.s.ms_phase[2] += sg.ms_sparsify;
    st_.s.ms_phase[3] += sg.ms_merge;
    pev_[k].reset();
  }
  pools_[0].release(s_);
  pools_[1].release(s_);
  work_.release(s_);
  SPAQR_HIP(hipStreamSynchronize(s_));
  st_.s.ms_factor = now_ms() - t0_;
}

template <typename T>
void Engine<T>::plan_fronts(StagePlan<T>& P) {
  const int k = k_;
  if (k != S_.L) begin_stage();
  Stager& up = stager_[stager_cur_];
  const StageSym& ss = S_.st[k];
  const int64_t nclu = ss.nclu;
  StageApply<T>& ap = ap_[k];
  auto slot_list = [&](const std::vector<int32_t>& cl, std::vector<int32_t>& out) {
    for (int32_t c : cl) out.insert(out.end(), slots_.begin() + slot_ptr_[c], slots_.begin() + slot_ptr_[c + 1]);
  };
  auto blk = [&](int32_t i, int32_t j) -> T* {
    const int64_t b = ss.all.find(i, j);
    return b < 0 ? nullptr : pool_ + boff_[b];
  };
  spaqr_stage_stats_t& sg = st_.stage[k];
  sg.stage = k;
  persist_mark_ = persist_.used();
  const double ff0 = st_.s.flops_front;
  {
    // the root separator (heap node 1) at the start of the stage
    const StageClusters& cl = S_.ord.stages[k];
    int64_t top = 0;
    for (int64_t c = 0; c < nclu; ++c)
      if (cl.node[c] == 1) top += size_[c];
    sg.top_separator = top;
    if (k == std::min(2, S_.L)) st_.s.top_separator = top;
  }
  d_flag_ = persist_.alloc_n<int>(1, s_);
  P.zero.push_back({d_flag_, (int64_t)sizeof(int)});

  // ------------------------------------------------------------ fronts
  std::unique_ptr<HostScope> hsub(new HostScope("host_pf_sizes"));
  const int64_t nf = (int64_t)ss.fronts.size();
  std::vector<int32_t> fm(nf), fn(nf), fnc(nf), fld(nf);
  std::vector<int64_t> ws_off(nf + 1, 0), vr_off(nf + 1, 0), rsj_off(nf + 1, 0), tau_off(nf + 1, 0);
  constexpr int VA = 16 / (int)sizeof(T);  // workspace rows start on 16-byte boundaries
  int max_m = 1;
  for (int64_t f = 0; f < nf; ++f) {
    const FrontSym& F = ss.fronts[f];
    int m = size_[F.cluster], nc = size_[F.cluster];
    for (int32_t i : F.n1) m += size_[i];
    for (int32_t j : F.cols) nc += size_[j];
    fm[f] = m;
    fn[f] = size_[F.cluster];
    fnc[f] = nc;
    // rows hold whole 16-column panels of the pivot block, so the trailing
    // update of a split front reads its V rows as aligned vectors in bounds
    fld[f] = std::max((nc + VA - 1) / VA * VA, (size_[F.cluster] + 15) / 16 * 16);
    ws_off[f + 1] = ws_off[f] + (int64_t)m * fld[f];
    vr_off[f + 1] = vr_off[f] + (int64_t)m * fn[f];
    rsj_off[f + 1] = rsj_off[f] + (int64_t)fn[f] * (nc - fn[f]);
    tau_off[f + 1] = tau_off[f] + fn[f];
    max_m = std::max(max_m, m);
    const double mm = m, nn = fn[f], kk = nc - fn[f];
    st_.s.flops_front += 2.0 * mm * nn * nn - 2.0 / 3.0 * nn * nn * nn + 4.0 * mm * nn * kk;
    st_.s.fronts++;
    sg.fronts++;
    sg.front_pivots += fn[f];
    sg.max_front_rows = std::max(sg.max_front_rows, m);
    sg.max_front_pivots = std::max(sg.max_front_pivots, fn[f]);
  }
  sg.flops_front = st_.s.flops_front - ff0;
  const int jbf = qr_panel_width(max_m, sizeof(T));
  SPAQR_REQUIRE(jbf > 0, SPAQR_ENOMEM, "front too tall for the LDS panel");
  P.jbf = jbf;
  T* W = work_.alloc_n<T>(std::max<int64_t>(1, ws_off[nf]), s_);
  // T factors of the 64-reflector blocks of the fronts that may be split
  // (those with more rows or trailing columns than the split thresholds)
  const bool mfma = tuning().trail_mfma != 0;
  std::vector<int64_t> tb_off(nf + 1, 0);
  for (int64_t f = 0; f < nf; ++f) {
    const bool may_split = fn[f] > 0 && (fm[f] > tuning().split_rows || fnc[f] - fn[f] >= tuning().split_cols);
    tb_off[f + 1] = tb_off[f] + (mfma && may_split ? (int64_t)(fn[f] + kWYBlock - 1) / kWYBlock * kWYBlock * kWYBlock : 0);
  }
  T* TB = tb_off[nf] > 0 ? work_.alloc_n<T>(tb_off[nf], s_) : nullptr;
  T* VR = persist_.alloc_n<T>(std::max<int64_t>(1, vr_off[nf]), s_);
  T* RSJ = persist_.alloc_n<T>(std::max<int64_t>(1, rsj_off[nf]), s_);
  T* TAU = persist_.alloc_n<T>(std::max<int64_t>(1, tau_off[nf]), s_);
  // compact-WY panel factors of every front (used by the forward apply)
  std::vector<int64_t> tp_off(nf + 1, 0);
  for (int64_t f = 0; f < nf; ++f) tp_off[f + 1] = tp_off[f] + (int64_t)((fn[f] + jbf - 1) / jbf) * jbf * jbf;
  T* TPF = persist_.alloc_n<T>(std::max<int64_t>(1, tp_off[nf]), s_);
  ap.jb = jbf;
  hsub.reset(new HostScope("host_pf_tiles"));
  for (size_t c = 0; c + 1 < ss.front_colour_ptr.size(); ++c) {
    typename StagePlan<T>::FrontColour fc;
    // slice width of this colour's split fronts
    {
      int mm = 0;
      for (int32_t oi = ss.front_colour_ptr[c]; oi < ss.front_colour_ptr[c + 1]; ++oi) {
        const int32_t f = ss.front_order[oi];
        if (fn[f] > 0 && (fm[f] > tuning().split_rows || fnc[f] - fn[f] >= tuning().split_cols))
          mm = std::max(mm, fm[f]);
      }
      if (mm > 0) {
        fc.trail_cw = trail_width(mm, sizeof(T));
        fc.trail_max_m = mm;
      }
    }
    // the colour's fronts in chunks planned in parallel (each chunk keeps
    // its own copy tiles; the other lists are joined in order, so the
    // descriptors are those of the sequential loop)
    struct Chunk {
      std::vector<CopyTile<T>> gather, scatter;
      std::vector<QRDesc<T>> qr;
      std::vector<TrailDesc<T>> trail;
      std::vector<WYBlock<T>> wyb;
      std::vector<WYTile<T>> wyt;
      int max_m = 1;
      double flops = 0.0, bytes = 0.0;
    };
    const int32_t o0 = ss.front_colour_ptr[c], o1 = ss.front_colour_ptr[c + 1];
    const int nfc = o1 - o0;
    const int nch = inner_pool_ && nfc >= 256 ? std::min(inner_pool_->size() + 1, nfc / 128) : 1;
    std::vector<Chunk> chunks(nch);
    const int trail_cw = fc.trail_cw;
    auto plan_chunk = [&](int q) {
      const int32_t ca = o0 + (int32_t)((int64_t)nfc * q / nch), cb = o0 + (int32_t)((int64_t)nfc * (q + 1) / nch);
      Chunk& C = chunks[q];
      size_t np = 0;
      for (int32_t oi = ca; oi < cb; ++oi) np += ss.fronts[ss.front_order[oi]].blk.size();
      C.gather.reserve(np);
      C.scatter.reserve(np);
      for (int32_t oi = ca; oi < cb; ++oi) {
        const int32_t f = ss.front_order[oi];
        const FrontSym& F = ss.fronts[f];
        T* Wf = W + ws_off[f];
        const int32_t nc = fnc[f], n = fn[f], ldw = fld[f];
        const size_t nr = 1 + F.n1.size(), ncl = 1 + F.cols.size();
        int ro = 0;
        for (size_t a = 0; a < nr; ++a) {
          int co = 0;
          const int32_t i = a == 0 ? F.cluster : F.n1[a - 1];
          const int64_t* brow = F.blk.data() + a * ncl;
          for (size_t b = 0; b < ncl; ++b) {
            const int32_t j = b == 0 ? F.cluster : F.cols[b - 1];
            if (size_[i] > 0 && size_[j] > 0) {
              T* blkp = brow[b] < 0 ? nullptr : pool_ + boff_[brow[b]];
              C.gather.push_back({blkp, Wf + (int64_t)ro * ldw + co, size_[i], size_[j], size_[j], ldw});
              if (a > 0 && b > 0) {
                SPAQR_REQUIRE(blkp != nullptr, SPAQR_EINVAL, "fill block missing from the stage pattern");
                C.scatter.push_back({Wf + (int64_t)ro * ldw + co, blkp, size_[i], size_[j], ldw, size_[j]});
              }
            }
            co += size_[j];
          }
          ro += size_[i];
        }
        if (n > 0) {
          const bool split = trail_cw > 0 && (fm[f] > tuning().split_rows || nc - n >= tuning().split_cols);
          C.qr.push_back({Wf, TAU + tau_off[f], TPF + tp_off[f], d_flag_, fm[f], n, split ? n : nc, ldw});
          if (split && mfma) {
            T* tb = TB + tb_off[f];
            for (int j0 = 0; j0 < n; j0 += kWYBlock)
              C.wyb.push_back({Wf, TAU + tau_off[f], tb + (int64_t)(j0 / kWYBlock) * kWYBlock * kWYBlock, fm[f], n, ldw,
                               j0});
            for (int c0 = n; c0 < nc; c0 += kWYBlock)
              C.wyt.push_back({Wf, tb, Wf, nullptr, fm[f], n, ldw, c0, std::min(kWYBlock, nc - c0), ldw});
          } else if (split) {
            for (int c0 = n; c0 < nc; c0 += trail_cw)
              C.trail.push_back({Wf, TPF + tp_off[f], Wf, nullptr, fm[f], n, ldw, c0, std::min(trail_cw, nc - c0), ldw});
          }
          C.max_m = std::max(C.max_m, fm[f]);
          const double mm = fm[f], nn = n, kk = nc - n;
          C.flops += 2.0 * mm * nn * nn - 2.0 / 3.0 * nn * nn * nn + 4.0 * mm * nn * kk;
          C.bytes += 2.0 * mm * nc * sizeof(T);
        }
      }
    };
    if (nch > 1) inner_pool_->run(nch, plan_chunk);
    else plan_chunk(0);
    for (Chunk& C : chunks) {
      fc.gather.push_back(std::move(C.gather));
      fc.scatter.push_back(std::move(C.scatter));
      append(fc.qr, C.qr);
      append(fc.trail, C.trail);
      append(fc.wyb, C.wyb);
      append(fc.wyt, C.wyt);
      fc.max_m = std::max(fc.max_m, C.max_m);
      fc.flops += C.flops;
      fc.bytes += C.bytes;
    }
    P.fronts.push_back(std::move(fc));
  }
  // pack factors column-major for the apply and build the apply descriptors
  hsub.reset(new HostScope("host_pf_apply"));
  {
    // the fronts with pivots in colour order; offsets of their row and
    // column slot lists and pack tiles first, then every list filled in
    // parallel chunks straight into the pinned staging buffers
    std::vector<int32_t> act;
    act.reserve(nf);
    std::vector<int64_t> rs_off(1, 0), cs_off(1, 0), pk_off(1, 0);
    ap.colour_ptr.assign(1, 0);
    for (size_t c = 0; c + 1 < ss.front_colour_ptr.size(); ++c) {
      int cmax = 0;
      double ffb = 0, fvb = 0, ffl = 0;
      for (int32_t oi = ss.front_colour_ptr[c]; oi < ss.front_colour_ptr[c + 1]; ++oi) {
        const int32_t f = ss.front_order[oi];
        const int32_t m = fm[f], n = fn[f], nc = fnc[f];
        if (n == 0) continue;
        act.push_back(f);
        rs_off.push_back(rs_off.back() + m);
        cs_off.push_back(cs_off.back() + (nc - n));
        pk_off.push_back(pk_off.back() + (nc > n ? 2 : 1));
        cmax = std::max(cmax, m);
        ap.max_bwd_rows = std::max(ap.max_bwd_rows, nc);
        ap.max_n = std::max(ap.max_n, n);
        ap.max_k = std::max(ap.max_k, nc - n);
        const double mm = m, nn = n, kk = nc - n, eb = sizeof(T);
        // forward: V below the diagonal + tau + row slots; x rows in and out
        ffb += (mm * nn - nn * (nn + 1) / 2 + nn) * eb + 4 * mm;
        fvb += 16 * mm;
        ffl += 4 * (mm * nn - nn * (nn - 1) / 2);
        // backward: R_ss upper triangle + R_sj + slots; x_s in/out, x_j in
        ap.bwd_fac_bytes += (nn * (nn + 1) / 2 + nn * kk) * eb + 4 * (nn + kk);
        ap.bwd_vec_bytes += 16 * nn + 8 * kk;
        ap.bwd_flops += nn * nn + 2 * nn * kk;
      }
      ap.colour_ptr.push_back((int64_t)act.size());
      ap.colour_max_m.push_back(cmax);
      ap.fwd_fac_bytes.push_back(ffb);
      ap.fwd_vec_bytes.push_back(fvb);
      ap.fwd_flops.push_back(ffl);
    }
    const int64_t na = (int64_t)act.size();
    hsub.reset(new HostScope("host_pf_upload"));
    Stager::Region rr{nullptr, nullptr, 0}, rc{nullptr, nullptr, 0};
    if (rs_off[na] > 0) rr = up.stage(persist_, (size_t)rs_off[na] * sizeof(int32_t), s_);
    if (cs_off[na] > 0) rc = up.stage(persist_, (size_t)cs_off[na] * sizeof(int32_t), s_);
    std::vector<ApFront<T>> af((size_t)na);
    P.pack.resize((size_t)pk_off[na]);
    const int nch = inner_pool_ && na >= 512 ? (int)std::min<int64_t>(inner_pool_->size() + 1, na / 256) : 1;
    auto fill = [&](int q) {
      const int64_t t0 = na * q / nch, t1 = na * (q + 1) / nch;
      auto put = [&](int32_t cl, int32_t*& dst) {
        const int64_t a0 = slot_ptr_[cl], a1 = slot_ptr_[cl + 1];
        std::memcpy(dst, slots_.data() + a0, (size_t)(a1 - a0) * sizeof(int32_t));
        dst += a1 - a0;
      };
      for (int64_t t = t0; t < t1; ++t) {
        const int32_t f = act[t];
        const FrontSym& F = ss.fronts[f];
        const int32_t m = fm[f], n = fn[f], nc = fnc[f];
        T* Wf = W + ws_off[f];
        P.pack[pk_off[t]] = {Wf, VR + vr_off[f], m, n, fld[f], m};
        if (nc > n) P.pack[pk_off[t] + 1] = {Wf + n, RSJ + rsj_off[f], n, nc - n, fld[f], n};
        int32_t* dr = static_cast<int32_t*>(rr.host) + rs_off[t];
        put(F.cluster, dr);
        for (int32_t i : F.n1) put(i, dr);
        if (rc.host) {
          int32_t* dc = static_cast<int32_t*>(rc.host) + cs_off[t];
          for (int32_t j : F.cols) put(j, dc);
        }
        af[t] = {VR + vr_off[f], RSJ + rsj_off[f], TAU + tau_off[f], TPF + tp_off[f],
                 static_cast<int32_t*>(rr.dev) + rs_off[t],
                 rc.dev ? static_cast<int32_t*>(rc.dev) + cs_off[t] : nullptr, m, n, nc - n, jbf};
      }
    };
    if (nch > 1) inner_pool_->run(nch, fill);
    else fill(0);
    if (rr.bytes) up.send(rr, s_);
    if (rc.bytes) up.send(rc, s_);
    ap.fronts = up.upload_held(persist_, af, s_);
    ap.nfronts = na;
    ap.h_fronts = std::move(af);
  }

  hsub.reset(new HostScope("host_pf_flush"));
  {
    std::vector<int> r0(size_.begin(), size_.end());
    r0.push_back(0);
    d_rank_ = up.upload_held(persist_, r0, s_);
  }
  up.flush(s_);
}

template <typename T>
void Engine<T>::plan_scale(StagePlan<T>& P) {
  const int k = k_;
  const StageSym& ss = S_.st[k];
  const int64_t nclu = ss.nclu;
  if (!ss.sparsify || !o_.scale) return;
  auto blk = [&](int32_t i, int32_t j) -> T* {
    const int64_t b = ss.all.find(i, j);
    return b < 0 ? nullptr : pool_ + boff_[b];
  };
  const std::vector<int32_t>& rem = ss.remaining;
  const int64_t ni = (int64_t)rem.size();
  const double fs0 = st_.s.flops_scale;
  st_.stage[k].sparsified = 1;
  std::vector<int32_t>& fidx = ib_.fidx;
  std::vector<int64_t>& u_off = ib_.u_off;
  std::vector<int64_t>& t_off = ib_.t_off;
  std::vector<int64_t>& p_off = ib_.p_off;
  fidx.assign(nclu, -1);
  u_off.assign(ni + 1, 0);
  t_off.assign(ni + 1, 0);
  p_off.assign(ni + 1, 0);
  int max_p = 1;
  for (int64_t t = 0; t < ni; ++t) {
    fidx[rem[t]] = (int32_t)t;
    const int64_t Pn = size_[rem[t]];
    u_off[t + 1] = u_off[t] + Pn * Pn;
    p_off[t + 1] = p_off[t] + Pn;
    max_p = std::max<int>(max_p, (int)Pn);
  }
  const int jbs = qr_panel_width(max_p, sizeof(T));
  SPAQR_REQUIRE(jbs > 0, SPAQR_ENOMEM, "interface too large for the LDS panel");
  P.jbs = jbs;
  P.max_p = max_p;
  for (int64_t t = 0; t < ni; ++t) {
    const int64_t Pn = size_[rem[t]];
    t_off[t + 1] = t_off[t] + ((Pn + jbs - 1) / jbs) * jbs * jbs;
    const double pp = Pn;
    st_.s.flops_scale += 4.0 / 3.0 * pp * pp * pp;
  }
  // the scaling QRs work row-major with rows padded to whole 16-column
  // panels (aligned vector reads of V by the trailing-update kernel)
  std::vector<int64_t> sw_off(ni + 1, 0);
  for (int64_t t = 0; t < ni; ++t) {
    const int64_t Pn = size_[rem[t]];
    sw_off[t + 1] = sw_off[t] + Pn * ((Pn + 15) / 16 * 16);
  }
  T* SW = work_.alloc_n<T>(std::max<int64_t>(1, sw_off[ni]), s_);
  T* VRU = ib_.vru = persist_.alloc_n<T>(std::max<int64_t>(1, u_off[ni]), s_);
  T* TAUU = ib_.tauu = persist_.alloc_n<T>(std::max<int64_t>(1, p_off[ni]), s_);
  T* TPAN = ib_.tpan = persist_.alloc_n<T>(std::max<int64_t>(1, t_off[ni]), s_);
  ib_.vq = persist_.alloc_n<T>(std::max<int64_t>(1, u_off[ni]), s_);
  ib_.tauq = persist_.alloc_n<T>(std::max<int64_t>(1, p_off[ni]), s_);
  int* FLAGS = ib_.flags = persist_.alloc_n<int>(std::max<int64_t>(1, ni), s_);
  P.zero.push_back({FLAGS, (int64_t)std::max<int64_t>(1, ni) * (int64_t)sizeof(int)});
  P.fac.resize(ni);
  for (int64_t t = 0; t < ni; ++t) {
    const int32_t p = rem[t], Pn = size_[p];
    const int32_t Pld = (Pn + 15) / 16 * 16;
    P.fac[t] = {VRU + u_off[t], TAUU + p_off[t], TPAN + t_off[t], FLAGS + t, Pn, 0, SW + sw_off[t], Pld, 0};
    if (Pn == 0) continue;
    T* src = blk(p, p);
    SPAQR_REQUIRE(src != nullptr, SPAQR_EINVAL, "interface without a diagonal block");
    P.sgather.push_back({src, SW + sw_off[t], Pn, Pn, Pn, Pld});
    P.sqr.push_back({SW + sw_off[t], TAUU + p_off[t], TPAN + t_off[t], FLAGS + t, Pn, Pn, Pn, Pld});
    P.spack.push_back({SW + sw_off[t], VRU + u_off[t], Pn, Pn, Pld, Pn});
  }
  for (int64_t i = 0; i < nclu; ++i)
    for (int64_t u = ss.post.rowptr[i]; u < ss.post.rowptr[i + 1]; ++u) {
      const int32_t j = ss.post.col[u];
      if (size_[i] == 0 || size_[j] == 0) continue;
      const int64_t b = ss.post_all[u];
      P.sblk.push_back({pool_ + boff_[b], size_[i], size_[j], fidx[i], fidx[j]});
      st_.s.flops_scale += 4.0 * size_[i] * size_[i] * size_[j] + (double)size_[i] * size_[j] * size_[j];
    }
  st_.stage[k].flops_scale = st_.s.flops_scale - fs0;
}

template <typename T>
void Engine<T>::plan_sparsify(StagePlan<T>& P) {
  const int k = k_;
  const StageSym& ss = S_.st[k];
  if (!ss.sparsify) return;
  if (!o_.scale) {
    plan_sparsify_unscaled(P);
    return;
  }
  Stager& up = stager_[stager_cur_];
  StageApply<T>& ap = ap_[k];
  auto slot_list = [&](const std::vector<int32_t>& cl, std::vector<int32_t>& out) {
    for (int32_t c : cl) out.insert(out.end(), slots_.begin() + slot_ptr_[c], slots_.begin() + slot_ptr_[c + 1]);
  };
  const std::vector<int32_t>& rem = ss.remaining;
  const int64_t ni = (int64_t)rem.size();
  const std::vector<int32_t>& fidx = ib_.fidx;
  const std::vector<int64_t>& u_off = ib_.u_off;
  const std::vector<int64_t>& p_off = ib_.p_off;
  T* VRU = ib_.vru;
  T* TAUU = ib_.tauu;
  T* VQ = ib_.vq;
  T* TAUQ = ib_.tauq;
  int* FLAGS = ib_.flags;
  // sparsification, colour by colour; CPQR workspaces: (colour, index,
  // offsets of C, the norms and the permutation)
  std::vector<std::array<int64_t, 5>> ws_at;
  int64_t wc_max = 0, wn_max = 0, wp_max = 0;
  for (size_t c = 0; c + 1 < ss.iface_colour_ptr.size(); ++c) {
    int64_t wc = 0, wn = 0, wp = 0;
    typename StagePlan<T>::SpColour col;
    for (int32_t oi = ss.iface_colour_ptr[c]; oi < ss.iface_colour_ptr[c + 1]; ++oi) {
      const IfaceSym& I = ss.ifaces[ss.iface_order[oi]];
      const int32_t p = I.cluster, Pn = size_[p];
      if (Pn == 0) continue;
      SpDesc<T> d{};
      d.nb = (int64_t)col.nb.size();
      int64_t mmax = 0;
      for (size_t q = 0; q < I.rowN.size(); ++q) {
        const int32_t i = I.rowN[q];
        col.nb.push_back({boff_[I.rowB[q]], i, Pn});
        mmax += size_[i];
      }
      for (size_t q = 0; q < I.colN.size(); ++q) {
        const int32_t j = I.colN[q];
        col.nb.push_back({boff_[I.colB[q]], j, size_[j]});
        mmax += size_[j];
      }
      d.nrow = (int32_t)I.rowN.size();
      d.ncol = (int32_t)I.colN.size();
      d.cluster = p;
      d.P = Pn;
      d.mmax = (int32_t)std::max<int64_t>(1, mmax);
      const int64_t t = fidx[p];
      d.vq = VQ + u_off[t];
      d.tauq = TAUQ + p_off[t];
      d.flag = FLAGS + t;
      d.pool = pool_;
      d.rank = d_rank_;
      d.eps = o_.eps;
      // the LDS/global kernels need a workspace; the register kernel needs
      // one only for its columns in global memory.  Offsets restart with
      // each colour: the colours run in stream order, so one region sized
      // for the largest colour serves them all
      if (!tuning().cpqr_reg || sparsify_reg_cpt(sizeof(T), Pn, d.mmax) == 0 ||
          sparsify_reg_global(sizeof(T), Pn, d.mmax)) {
        ws_at.push_back({(int64_t)P.sp.size(), (int64_t)col.sd.size(), wc, wn, wp});
        wc += (int64_t)(Pn <= 64 ? 65 : Pn) * d.mmax;
        wn += d.mmax;
        wp += 2 * (int64_t)d.mmax;
      }
      col.sd.push_back(d);
    }
    wc_max = std::max(wc_max, wc);
    wn_max = std::max(wn_max, wn);
    wp_max = std::max(wp_max, wp);
    P.sp.push_back(std::move(col));
  }
  if (!ws_at.empty()) {
    T* WC = work_.alloc_n<T>((size_t)wc_max, s_);
    double* WN = work_.alloc_n<double>((size_t)wn_max, s_);
    int32_t* WP = work_.alloc_n<int32_t>((size_t)wp_max, s_);
    for (const auto& w : ws_at) {
      SpDesc<T>& d = P.sp[w[0]].sd[w[1]];
      d.C = WC + w[2];
      d.nrm = WN + w[3];
      d.perm = WP + w[4];
    }
  }
  // apply descriptors of the interfaces; those of at most 64 unknowns get
  // their dense forward and backward operators
  std::vector<ApIface<T>> ai;
  std::vector<int32_t> sl;
  std::vector<int64_t> sl_off;
  int64_t dense_elems = 0;
  const int dmax = ap.dense_max = tuning().iface_dense;
  for (int64_t t = 0; t < ni; ++t) {
    const int64_t Pn = size_[rem[t]];
    if (Pn > 0 && Pn <= dmax) dense_elems += Pn * Pn;
  }
  T* MF = persist_.alloc_n<T>(std::max<int64_t>(1, dense_elems), s_);
  T* MB = persist_.alloc_n<T>(std::max<int64_t>(1, dense_elems), s_);
  int64_t dense_off = 0;
  for (int64_t t = 0; t < ni; ++t) {
    const int32_t p = rem[t], Pn = size_[p];
    if (Pn == 0) continue;
    sl_off.push_back((int64_t)sl.size());
    slot_list(std::vector<int32_t>{p}, sl);
    T* mf = nullptr;
    T* mb = nullptr;
    if (Pn <= dmax) {
      mf = MF + dense_off;
      mb = MB + dense_off;
      dense_off += (int64_t)Pn * Pn;
    }
    ai.push_back({VRU + u_off[t], TAUU + p_off[t], VQ + u_off[t], TAUQ + p_off[t], nullptr, d_rank_ + p,
                  FLAGS + t, mf, mb, Pn, 0});
    ap.max_p = std::max(ap.max_p, (int)Pn);
  }
  int32_t* dsl = up.upload_held(persist_, sl, s_);
  for (size_t t = 0; t < ai.size(); ++t) ai[t].slots = dsl + sl_off[t];
  // interfaces with dense operators first (dense-operator apply)
  std::stable_partition(ai.begin(), ai.end(), [dmax](const ApIface<T>& q) { return q.P <= dmax; });
  for (const ApIface<T>& q : ai)
    if (q.P <= dmax) {
      ap.nifaces_small++;
      ap.dense_max_p = std::max(ap.dense_max_p, (int)q.P);
    }
  ap.ifaces = up.upload_held(persist_, ai, s_);
  up.flush(s_);
  ap.nifaces = (int64_t)ai.size();
  P.form.assign(ai.begin(), ai.begin() + ap.nifaces_small);
  st_.s.interfaces_sparsified += (int64_t)ai.size();
  ap.h_ifaces = std::move(ai);
}

// Sparsification without scaling (Section 2.5): per colour, one workgroup per
// interface (k_sparsify_unscaled), which also writes the interface's dense
// forward and backward apply operators.  The FP64 workspaces of one colour
// are reused by the next (colours run in stream order).
template <typename T>
void Engine<T>::plan_sparsify_unscaled(StagePlan<T>& P) {
  const int k = k_;
  const StageSym& ss = S_.st[k];
  Stager& up = stager_[stager_cur_];
  StageApply<T>& ap = ap_[k];
  auto slot_list = [&](const std::vector<int32_t>& cl, std::vector<int32_t>& out) {
    for (int32_t c : cl) out.insert(out.end(), slots_.begin() + slot_ptr_[c], slots_.begin() + slot_ptr_[c + 1]);
  };
  const std::vector<int32_t>& rem = ss.remaining;
  const int64_t ni = (int64_t)rem.size();
  st_.stage[k].sparsified = 1;
  std::vector<int32_t> fidx(ss.nclu, -1);
  std::vector<int64_t> op_off(ni + 1, 0);
  for (int64_t t = 0; t < ni; ++t) {
    fidx[rem[t]] = (int32_t)t;
    op_off[t + 1] = op_off[t] + (int64_t)size_[rem[t]] * size_[rem[t]];
  }
  int* FLAGS = persist_.alloc_n<int>(std::max<int64_t>(1, ni), s_);
  P.zero.push_back({FLAGS, (int64_t)std::max<int64_t>(1, ni) * (int64_t)sizeof(int)});
  T* MF = persist_.alloc_n<T>(std::max<int64_t>(1, op_off[ni]), s_);
  T* MB = persist_.alloc_n<T>(std::max<int64_t>(1, op_off[ni]), s_);
  // descriptors colour by colour; workspace offsets restart with each colour
  int64_t ws_max = 1;
  std::vector<std::vector<int64_t>> ws_at(ss.iface_colour_ptr.size());
  for (size_t c = 0; c + 1 < ss.iface_colour_ptr.size(); ++c) {
    typename StagePlan<T>::SpuColour col;
    int64_t wo = 0;
    for (int32_t oi = ss.iface_colour_ptr[c]; oi < ss.iface_colour_ptr[c + 1]; ++oi) {
      const IfaceSym& I = ss.ifaces[ss.iface_order[oi]];
      const int32_t p = I.cluster, Pn = size_[p];
      if (Pn == 0) continue;
      SPAQR_REQUIRE(Pn <= kSpuMaxP, SPAQR_EINVAL, "interface too large for the sparsification without scaling");
      SPAQR_REQUIRE((int64_t)(I.rowN.size() + I.colN.size()) <= kSpuMaxNbr, SPAQR_EINVAL,
                    "interface with too many neighbour blocks for the sparsification without scaling");
      SpuDesc<T> d{};
      d.nb = (int64_t)col.nb.size();
      int64_t mr = 0, mc = 0;
      for (size_t q = 0; q < I.rowN.size(); ++q) {
        col.nb.push_back({boff_[I.rowB[q]], I.rowN[q], Pn});
        mr += size_[I.rowN[q]];
      }
      for (size_t q = 0; q < I.colN.size(); ++q) {
        col.nb.push_back({boff_[I.colB[q]], I.colN[q], size_[I.colN[q]]});
        mc += size_[I.colN[q]];
      }
      const int64_t t = fidx[p];
      d.pool = pool_;
      d.rank = d_rank_;
      d.flag = FLAGS + t;
      d.mf = MF + op_off[t];
      d.mb = MB + op_off[t];
      d.ws = nullptr;
      d.eps = o_.eps;
      const int64_t bpp = I.ppB;
      SPAQR_REQUIRE(bpp >= 0, SPAQR_EINVAL, "interface without a diagonal block");
      d.app = boff_[bpp];
      d.nrow = (int32_t)I.rowN.size();
      d.ncol = (int32_t)I.colN.size();
      d.cluster = p;
      d.P = Pn;
      d.mr_max = (int32_t)mr;
      d.mc_max = (int32_t)mc;
      ws_at[c].push_back(wo);
      wo += (sparsify_unscaled_ws(Pn, (int)mr, (int)mc) + 31) / 32 * 32;
      col.sd.push_back(d);
    }
    ws_max = std::max(ws_max, wo);
    P.spu.push_back(std::move(col));
  }
  double* WS = work_.alloc_n<double>((size_t)ws_max, s_);
  for (size_t c = 0; c < P.spu.size(); ++c)
    for (size_t q = 0; q < P.spu[c].sd.size(); ++q) P.spu[c].sd[q].ws = WS + ws_at[c][q];
  // every interface applies through its dense operators
  std::vector<ApIface<T>> ai;
  std::vector<int32_t> sl;
  std::vector<int64_t> sl_off;
  ap.dense_max = INT32_MAX;
  for (int64_t t = 0; t < ni; ++t) {
    const int32_t p = rem[t], Pn = size_[p];
    if (Pn == 0) continue;
    sl_off.push_back((int64_t)sl.size());
    slot_list(std::vector<int32_t>{p}, sl);
    ai.push_back({nullptr, nullptr, nullptr, nullptr, nullptr, d_rank_ + p, FLAGS + t, MF + op_off[t], MB + op_off[t],
                  Pn, 0});
    ap.max_p = std::max(ap.max_p, (int)Pn);
    ap.dense_max_p = std::max(ap.dense_max_p, (int)Pn);
  }
  int32_t* dsl = up.upload_held(persist_, sl, s_);
  for (size_t t = 0; t < ai.size(); ++t) ai[t].slots = dsl + sl_off[t];
  ap.nifaces_small = (int64_t)ai.size();
  ap.ifaces = up.upload_held(persist_, ai, s_);
  up.flush(s_);
  ap.nifaces = (int64_t)ai.size();
  st_.s.interfaces_sparsified += (int64_t)ai.size();
  ap.h_ifaces = std::move(ai);
}

template <typename T>
void Engine<T>::readback_ops(std::vector<IntCopy>& ops, int32_t base) const {
  const int32_t nclu = (int32_t)S_.st[k_].nclu;
  ops.push_back({d_rank_, base, nclu});
  ops.push_back({d_flag_, base + nclu, 1});
  ops.push_back({d_zcol_, base + nclu + 1, 1});
}

template <typename T>
void Engine<T>::finish(MergePlan<T>& mp) {
  const int k = k_;
  const StageSym& ss = S_.st[k];
  const int64_t nclu = ss.nclu;
  StageApply<T>& ap = ap_[k];
  if (rb_[nclu + 1] != 0 || rb_[nclu] != 0) {
    // recorded, not thrown: the other factorizations of a batch carry on
    err_ = rb_[nclu + 1] != 0 ? SPAQR_EINVAL : SPAQR_ESINGULAR;
    err_msg_ = rb_[nclu + 1] != 0 ? "A has a zero column" : "a front produced an exactly zero R_ss diagonal";
    k_ = 0;
    return;
  }
  st_.stage_sizes[k].assign(rb_, rb_ + nclu);
  spaqr_stage_stats_t& sg = st_.stage[k];
  sg.factor_bytes = (int64_t)(persist_.used() - persist_mark_);
  if (ss.sparsify) {
    const double eb = sizeof(T);
    std::vector<int32_t> iidx(nclu, -1);
    for (size_t t = 0; t < ss.ifaces.size(); ++t) iidx[ss.ifaces[t].cluster] = (int32_t)t;
    double sp_flops = 0.0, sp_bytes = 0.0, ul_flops = 0.0, ul_bytes = 0.0;
    for (size_t t = 0; t < ss.ifaces.size(); ++t) {
      const IfaceSym& I = ss.ifaces[t];
      const int32_t p = I.cluster;
      const double P = size_[p], r = rb_[p];
      if (P == 0) continue;
      if (P <= ap.dense_max) {
        // dense operators Q^T U^T and R^{-1} Q
        ap.if_fwd_fac_bytes += P * P * eb + 4 * P;
        ap.if_bwd_fac_bytes += P * P * eb + 4 * P;
        ap.if_fwd_flops += 2 * P * P;
        ap.if_bwd_flops += 2 * P * P;
      } else {
        // U below the diagonal + tau, then the kept reflectors of Q
        const double qel = r < P ? (P * r - r * (r - 1) / 2) : 0.0;
        ap.if_fwd_fac_bytes += (P * (P - 1) / 2 + P + qel + (r < P ? r : 0)) * eb + 4 * P;
        ap.if_bwd_fac_bytes += (P * (P + 1) / 2 + qel + (r < P ? r : 0)) * eb + 4 * P;
        ap.if_fwd_flops += 4 * (P * (P + 1) / 2 + qel);
        ap.if_bwd_flops += P * P + 4 * qel;
      }
      ap.if_vec_bytes += 16 * P;
      // CPQR work, the method's own count: the columns of C are the
      // neighbours' current unknowns (a neighbour of an earlier colour
      // already has its new rank); Householder QR of the r accepted pivot
      // columns of the |p| x m matrix with its trailing update,
      // 4|p|mr - 2r^2(|p| + m) + 4/3 r^3, plus one norm update per column
      // and step, m r
      double mr = 0.0, mc = 0.0;
      for (int32_t q : I.rowN) mr += ss.ifaces[iidx[q]].colour < I.colour ? rb_[q] : size_[q];
      for (int32_t q : I.colN) mc += ss.ifaces[iidx[q]].colour < I.colour ? rb_[q] : size_[q];
      const double m = mr + mc;
      const double fl = 4.0 * P * m * r - 2.0 * r * r * (P + m) + 4.0 / 3.0 * r * r * r + m * r;
      if (!o_.scale) {
        // without scaling (Section 2.5), on top of the CPQR: bidiagonalization
        // of the (P + m_r) x P matrix A_p for sigma_min, 4(P + m_r)P^2 -
        // 4/3 P^3; sigma A_pp^T A_pn, 2 P^2 m_c; and when r < P (f = P - r):
        // A_pp Q and the backward operator's Q, each 4P(Pr - r(r-1)/2); the QR
        // of the f columns, 2Pf^2 - 2/3 f^3, with its reflectors applied to
        // the r + m_c other columns and to the forward operator's P columns,
        // 4(r + m_c + P)(Pf - f(f-1)/2); the backward operator's triangular
        // solves, P f^2
        const double f = P - r;
        double ul = 4.0 * (P + mr) * P * P - 4.0 / 3.0 * P * P * P + 2.0 * P * P * mc + fl;
        if (f > 0)
          ul += 8.0 * P * (P * r - r * (r - 1) / 2) + 2.0 * P * f * f - 2.0 / 3.0 * f * f * f +
                4.0 * (r + mc + P) * (P * f - f * (f - 1) / 2) + P * f * f;
        ul_flops += ul;
        // blocks read once and written once, both operators written
        ul_bytes += (P * P + P * m) * eb * 2 + (f > 0 ? 2 * P * P * eb : 0.0);
      }
      sp_flops += fl;
      st_.s.flops_sparsify += fl;
      sg.flops_sparsify += fl;
      sg.interfaces++;
      sg.iface_unknowns_in += (int64_t)P;
      sg.iface_unknowns_out += (int64_t)r;
      sg.nbr_cols += (int64_t)m;
      sg.max_nbr_cols = std::max(sg.max_nbr_cols, (int32_t)m);
      st_.ifaces[k].insert(st_.ifaces[k].end(), {p, (int32_t)P, (int32_t)m, (int32_t)r});
      sp_bytes += (P * m + (r < P ? r * m : 0.0)) * eb;
    }
    if (o_.scale) prof_add("sparsify", sp_flops, sp_bytes);
    else prof_add("sparsify_unscaled", ul_flops, ul_bytes);
    std::vector<int32_t> ps;
    for (size_t t = 1; t < st_.ifaces[k].size(); t += 4) ps.push_back(st_.ifaces[k][t]);
    if (!ps.empty()) {
      std::sort(ps.begin(), ps.end());
      const size_t np = ps.size();
      sg.iface_size_q1 = ps[np / 4];
      sg.iface_size_median = ps[np / 2];
      sg.iface_size_q3 = ps[(3 * np) / 4];
      sg.iface_size_max = ps.back();
    }
  }
  if (k == 1) {
    k_ = 0;
    complete();
    return;
  }
  // ------------------------------------------------ merge to stage k - 1
  const StageSym& s2 = S_.st[k - 1];
  const std::vector<int64_t>& par = S_.ord.stages[k].parent;
  const std::vector<int32_t>& rank = st_.stage_sizes[k];
  const int64_t n2 = s2.nclu;
  std::vector<int32_t> size2(n2, 0);
  std::vector<int32_t> off(ss.nclu, 0);
  for (int64_t c = 0; c < ss.nclu; ++c) {
    if (par[c] < 0) continue;
    off[c] = size2[par[c]];
    size2[par[c]] += rank[c];
  }
  // slot lists of the merged clusters: children's surviving slots in order
  std::vector<int64_t> sp2(n2 + 1, 0);
  for (int64_t Pc = 0; Pc < n2; ++Pc) sp2[Pc + 1] = sp2[Pc] + size2[Pc];
  std::vector<int32_t> sl2(sp2[n2]);
  for (int64_t c = 0; c < ss.nclu; ++c) {
    if (par[c] < 0) continue;
    std::copy(slots_.begin() + slot_ptr_[c], slots_.begin() + slot_ptr_[c] + rank[c],
              sl2.begin() + sp2[par[c]] + off[c]);
  }
  // new pool
  std::vector<int64_t> boff2(s2.all.size() + 1, 0);
  for (int64_t i = 0; i < n2; ++i)
    for (int64_t t = s2.all.rowptr[i]; t < s2.all.rowptr[i + 1]; ++t)
      boff2[t + 1] = boff2[t] + (int64_t)size2[i] * size2[s2.all.col[t]];
  DevArena& pa = pools_[(k - 1) & 1];
  pa.reset();
  T* pool2 = pa.alloc_n<T>(std::max<int64_t>(1, boff2.back()), s_);
  // the new pool starts at zero (absent sub-blocks), then every child block
  // lands in its own sub-block of the parent block: disjoint destinations
  mp.zero.push_back({pool2, std::max<int64_t>(1, boff2.back()) * (int64_t)sizeof(T)});
  // the block copies, by chunks of block rows planned in parallel
  const int64_t nrows = ss.nclu, nblk = ss.post.rowptr[nrows];
  const int nch = inner_pool_ && nblk >= 65536 ? (int)std::min<int64_t>(inner_pool_->size() + 1, nblk / 16384) : 1;
  mp.tiles.assign(nch, {});
  auto tiles_of = [&](int q) {
    std::vector<CopyTile<T>>& out = mp.tiles[q];
    // block rows [row_at(q), row_at(q + 1)): the first row whose blocks
    // start at or after the chunk's share of the blocks
    auto row_at = [&](int c) -> int64_t {
      if (c == 0) return 0;
      if (c == nch) return nrows;
      return std::lower_bound(ss.post.rowptr.begin(), ss.post.rowptr.begin() + nrows + 1, nblk * c / nch) -
             ss.post.rowptr.begin();
    };
    const int64_t i0 = row_at(q), i1 = row_at(q + 1);
    out.reserve((size_t)(ss.post.rowptr[i1] - ss.post.rowptr[i0]));
    for (int64_t i = i0; i < i1; ++i)
      for (int64_t u = ss.post.rowptr[i]; u < ss.post.rowptr[i + 1]; ++u) {
        const int32_t j = ss.post.col[u];
        if (rank[i] == 0 || rank[j] == 0) continue;
        const int32_t Qc = (int32_t)par[j];
        const int64_t B = ss.post_next[u];
        SPAQR_REQUIRE(B >= 0, SPAQR_EINVAL, "merged block missing from the next stage pattern");
        const int64_t b = ss.post_all[u];
        out.push_back({pool_ + boff_[b], pool2 + boff2[B] + (int64_t)off[i] * size2[Qc] + off[j], rank[i], rank[j],
                       size_[j], size2[Qc]});
      }
  };
  if (nch > 1) inner_pool_->run(nch, tiles_of);
  else tiles_of(0);
  pool_ = pool2;
  boff_.swap(boff2);
  size_.swap(size2);
  slot_ptr_.swap(sp2);
  slots_.swap(sl2);
  k_ = k - 1;
}

// ------------------------------------------------------------ batch driver
// Launch lists of several factorizations (same precision, same stream)
// concatenated phase by phase: zero fills, then the fronts colour by colour
// (gather, QR, scatter), the factor packing, the scaling (gather, QR, pack,
// block update), the sparsification colour by colour and the dense interface
// operators; after one synchronization every factorization reads its ranks
// and the merges run as one zero fill and one copy launch.
struct BatchCtx {
  Stager st[2];
  DevArena work[2] = {DevArena(size_t(16) << 20), DevArena(size_t(16) << 20)};
  int cur = 0;
  std::unique_ptr<HostPool> pool;  // per-problem planning of a batch, in parallel
  hipEvent_t ev = nullptr;          // end of the enqueued part of the current stage
  std::shared_ptr<PhaseEvents> pe;  // phase events of the current stage
  PinnedChunk rb;                   // ranks and flags of the current stage, all problems
  int32_t team_err_at = -1;         // index in rb of the team CPQR timeout flag
  BatchCtx() = default;
  BatchCtx(const BatchCtx&) = delete;
  BatchCtx& operator=(const BatchCtx&) = delete;
  ~BatchCtx() {
    if (ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    pinned_release(rb);
  }
  void begin() {
    cur ^= 1;
    st[cur].reset();
    work[cur].reset();
  }
  HostPool* host_pool() {
    if (!pool) pool.reset(new HostPool(host_pool_threads()));
    return pool.get();
  }
  void each(size_t n, const std::function<void(int)>& fn) {
    if (n > 1 && !pool) {
      pool.reset(new HostPool(host_pool_threads()));
    }
    if (pool) pool->run((int)n, fn);
    else
      for (size_t i = 0; i < n; ++i) fn((int)i);
  }
};


static void launch_zero_ops(const std::vector<ZeroOp>& ops, Stager& up, DevArena& wk, hipStream_t s) {
  if (ops.empty()) return;
  std::vector<ZeroDesc> zd;
  int64_t blocks = 0;
  for (const ZeroOp& o : ops) {
    const int64_t words = (o.bytes + 3) / 4;
    if (words <= 0) continue;
    zd.push_back({static_cast<uint32_t*>(o.p), words, blocks});
    blocks += (words + kZeroWordsPerBlock - 1) / kZeroWordsPerBlock;
  }
  ZeroDesc* d = up.upload(wk, zd, s);
  launch_zero(d, (int64_t)zd.size(), blocks, s);
}

// QR descriptors grouped by the register-kernel plan of each factorization,
// so that every group shares a panel width: (jb, rows-per-thread class).
template <typename T>
static void launch_qr_groups(std::vector<std::pair<int, std::vector<QRDesc<T>>>>& parts, const char* prof_name,
                             double flops, double bytes, Stager& up, DevArena& wk, hipStream_t s) {
  std::map<std::pair<int, int>, std::pair<int, std::vector<QRDesc<T>>>> groups;
  for (auto& pr : parts) {
    if (pr.second.empty()) continue;
    int mm = 1;
    for (const QRDesc<T>& q : pr.second) mm = std::max(mm, (int)q.m);
    const int jb = pr.first;
    const int cls = mm <= 256 ? 1 : (mm <= 512 ? 2 : (mm <= 1024 ? 4 : 8 + mm));
    auto& g = groups[{jb, cls}];
    g.first = std::max(g.first, mm);
    append(g.second, pr.second);
  }
  if (groups.empty()) return;
  ProfScope ps(prof_name, s, flops, bytes);
  for (auto& kv : groups) {
    QRDesc<T>* d = up.upload(wk, kv.second.second, s);
    launch_qr<T>(d, (int64_t)kv.second.second.size(), kv.first.first, kv.second.first, s);
  }
}

// The concatenation of get(0), get(1), ... uploaded in one copy; large lists
// are packed into the pinned staging buffer by the planning threads.
template <typename X, typename Get>
static X* upload_concat(BatchCtx& bx, Stager& up, DevArena& wk, size_t ne, Get get, hipStream_t s,
                        int64_t* count) {
  std::vector<size_t> off(ne + 1, 0);
  for (size_t e = 0; e < ne; ++e) off[e + 1] = off[e] + get(e).size();
  *count = (int64_t)off[ne];
  if (off[ne] == 0) return nullptr;
  Stager::Region r;
  {
    HostScope hs("host_upload_stage");
    r = up.stage(wk, off[ne] * sizeof(X), s);
  }
  X* h = static_cast<X*>(r.host);
  auto put = [&](int e) {
    const std::vector<X>& v = get(e);
    if (!v.empty()) std::memcpy(h + off[e], v.data(), v.size() * sizeof(X));
  };
  {
    HostScope hs("host_upload_pack");
    if (ne > 1 && off[ne] * sizeof(X) > (size_t(1) << 20)) bx.each(ne, put);
    else
      for (size_t e = 0; e < ne; ++e) put((int)e);
  }
  HostScope hs("host_upload_send");
  up.send(r, s);
  return static_cast<X*>(r.dev);
}

// transpose: the lists hold transposing packs only, else plain copies only
// bytes a list of copies must move (read and write, or write for a fill)
template <typename T>
static double copy_bytes(const std::vector<CopyTile<T>>& tiles) {
  double b = 0.0;
  for (const CopyTile<T>& c : tiles) b += (c.src ? 2.0 : 1.0) * c.rows * (double)c.cols * sizeof(T);
  return b;
}

// (profiled under "copy" and under the name of the copy's role)
template <typename T, typename Get>
static void copy_concat(BatchCtx& bx, Stager& up, DevArena& wk, size_t ne, Get get, bool transpose, hipStream_t s,
                        const char* role) {
  int64_t n = 0;
  CopyTile<T>* d = upload_concat<CopyTile<T>>(bx, up, wk, ne, get, s, &n);
  if (n <= 0) return;
  double by = 0.0;
  if (prof_wants("copy") || prof_wants(role))
    for (size_t e = 0; e < ne; ++e) by += copy_bytes<T>(get(e));
  ProfScope ps("copy", s, 0.0, by);
  ProfScope pr(role, s, (double)n, by);
  launch_copy<T>(d, n, transpose, s);
}

template <typename T>
static void copy_batch(const std::vector<CopyTile<T>>& tiles, bool transpose, Stager& up, DevArena& wk,
                       hipStream_t s, const char* role) {
  if (tiles.empty()) return;
  CopyTile<T>* d = up.upload(wk, tiles, s);
  const double by = prof_wants("copy") || prof_wants(role) ? copy_bytes<T>(tiles) : 0.0;
  ProfScope ps("copy", s, 0.0, by);
  ProfScope pr(role, s, (double)tiles.size(), by);
  launch_copy<T>(d, (int64_t)tiles.size(), transpose, s);
}

template <typename T>
static void sparsify_batch(std::vector<SpDesc<T>>& sd, const std::vector<SpNbr>& nb, Stager& up, DevArena& wk,
                           hipStream_t s, int* team_err) {
  if (sd.empty()) return;
  int max_nb = 0, max_pc = 1;
  for (const SpDesc<T>& q : sd) {
    max_nb = std::max(max_nb, q.nrow + q.ncol);
    max_pc = std::max<int>(max_pc, q.P);
  }
  SpNbr* dnb = nullptr;
  if constexpr (std::is_same<T, float>::value) {
    // FP32 interfaces of at most 64 unknowns whose columns fit one
    // workgroup: the downdated-norm CPQR, all of them in one launch, the
    // largest first
    if (tuning().cpqr_dd) {
      const auto dd_end = std::stable_partition(sd.begin(), sd.end(), [](const SpDesc<T>& q) {
        return q.P >= 1 && q.P <= 64 && q.mmax <= sparsify_dd_capacity(q.P);
      });
      if (dd_end != sd.begin()) {
        std::vector<SpDesc<T>> dd(sd.begin(), dd_end);
        sd.erase(sd.begin(), dd_end);
        std::stable_sort(dd.begin(), dd.end(), [](const SpDesc<T>& x, const SpDesc<T>& y) {
          return (int64_t)x.P * x.mmax > (int64_t)y.P * y.mmax;
        });
        int lc_rows = 0;
        for (const SpDesc<T>& q : dd) lc_rows = std::max(lc_rows, sparsify_dd_lc_rows(q.P, q.mmax));
        SpDesc<T>* ddd = up.upload(wk, dd, s);
        dnb = up.upload(wk, nb, s);
        ProfScope ps("sparsify", s, 0.0, 0.0);
        launch_sparsify_dd(ddd, (int64_t)dd.size(), dnb, max_nb, lc_rows, s);
      }
      if (sd.empty()) return;
    }
    // FP32 interfaces of 65-896 unknowns: a team of co-resident workgroups
    // per interface, the interfaces packed into launches of at most the
    // device's co-resident workgroups, the largest first.  (Measured: on the
    // 64^3 grid the team kernel takes 3.6 s of sparsification against 5.1 s
    // for the cooperative one; for wide interfaces of at most 64 unknowns the
    // cooperative kernel is faster, 34 against 41 ms per 1024^2 problem.)
    if (tuning().cpqr_team) {
      const int cap = sparsify_team_capacity(max_nb);
      const auto tm_end = std::stable_partition(sd.begin(), sd.end(), [&](const SpDesc<T>& q) {
        const int nb_q = sparsify_team_blocks(q.P, q.mmax);
        const bool wide = q.P > 64 || (tuning().cpqr_team == 2 && q.mmax >= 16384);
        return wide && nb_q > 0 && nb_q <= cap;
      });
      if (tm_end != sd.begin()) {
        std::vector<SpDesc<T>> tm(sd.begin(), tm_end);
        sd.erase(sd.begin(), tm_end);
        std::stable_sort(tm.begin(), tm.end(), [](const SpDesc<T>& x, const SpDesc<T>& y) {
          return sparsify_team_blocks(x.P, x.mmax) > sparsify_team_blocks(y.P, y.mmax);
        });
        struct TeamLaunch {
          size_t begin, end;
          int blocks;
        };
        std::vector<TeamLaunch> launches;
        std::vector<CoopItem> items;
        int max_blocks = 0;
        for (size_t t = 0; t < tm.size(); ++t) {
          const int nb_t = sparsify_team_blocks(tm[t].P, tm[t].mmax);
          if (launches.empty() || launches.back().blocks + nb_t > cap) launches.push_back({t, t, 0});
          items.push_back({launches.back().blocks, nb_t});
          launches.back().blocks += nb_t;
          launches.back().end = t + 1;
          max_blocks = std::max(max_blocks, launches.back().blocks);
        }
        SpDesc<T>* dtm = up.upload(wk, tm, s);
        CoopItem* ditems = up.upload(wk, items, s);
        if (!dnb) dnb = up.upload(wk, nb, s);
        int* sync = wk.alloc_n<int>(2 * tm.size(), s);
        char* cand = wk.alloc_n<char>(sparsify_team_cand_bytes(max_blocks), s);
        launch_zero_ops({{sync, (int64_t)(2 * tm.size() * sizeof(int))}}, up, wk, s);
        for (const TeamLaunch& L : launches) {
          ProfScope ps("sparsify", s, 0.0, 0.0);
          if (!launch_sparsify_team(dtm + L.begin, ditems + L.begin, (int)(L.end - L.begin), L.blocks, dnb, max_nb,
                                    sync + 2 * L.begin, cand, max_blocks, team_err, s))
            throw Error(SPAQR_EDEVICE, "team CPQR no longer fits the device");
        }
      }
      if (sd.empty()) return;
    }
  }
  // interfaces whose columns fit in registers: register CPQR, one launch per
  // (row class, columns per thread) when one shape does not fit all
  const auto nreg_end = std::stable_partition(
      sd.begin(), sd.end(),
      [](const SpDesc<T>& q) { return tuning().cpqr_reg && sparsify_reg_cpt(sizeof(T), q.P, q.mmax) > 0; });
  const int64_t nreg = nreg_end - sd.begin();
  int preg = 1, mreg = 1;
  for (int64_t t = 0; t < nreg; ++t) {
    preg = std::max<int>(preg, sd[t].P);
    mreg = std::max<int>(mreg, sd[t].mmax);
  }
  std::vector<std::array<int64_t, 4>> groups;  // begin, end, pmax, mmax
  if (nreg > 0 && sparsify_reg_cpt(sizeof(T), preg, mreg) > 0 && !sparsify_reg_global(sizeof(T), preg, mreg)) {
    groups.push_back({0, nreg, preg, mreg});
  } else if (nreg > 0) {
    auto pcls = [](int Pv) { return Pv <= 16 ? 0 : (Pv <= 32 ? 1 : 2); };
    std::stable_sort(sd.begin(), sd.begin() + nreg,
                     [&](const SpDesc<T>& x, const SpDesc<T>& y) { return pcls(x.P) < pcls(y.P); });
    for (int64_t b = 0; b < nreg;) {
      int64_t e = b;
      int pm = 1, mm = 1;
      while (e < nreg && pcls(sd[e].P) == pcls(sd[b].P)) {
        pm = std::max<int>(pm, sd[e].P);
        mm = std::max<int>(mm, sd[e].mmax);
        ++e;
      }
      groups.push_back({b, e, pm, mm});
      b = e;
    }
  }
  // interfaces beyond one workgroup: the cooperative CPQR (64 * cpt columns
  // per one-wave workgroup), interfaces packed into launches whose workgroups
  // can all be co-resident, the longest factorizations first; cpt is the
  // smallest that needs the fewest launches
  struct CoopLaunch {
    int64_t begin, end;
    int blocks, kmax;
  };
  std::vector<CoopLaunch> coop;
  std::vector<CoopItem> items;
  int coop_cpt = 0, coop_maxp = 1, coop_maxnb = 0, coop_blocks = 1;
  int64_t ncoop = 0;
  if ((int64_t)sd.size() > nreg && tuning().cpqr_coop) {
    auto kmax_of = [](const SpDesc<T>& q) { return std::min<int>(q.P, q.mmax); };
    std::stable_sort(sd.begin() + nreg, sd.end(),
                     [&](const SpDesc<T>& x, const SpDesc<T>& y) { return kmax_of(x) > kmax_of(y); });
    for (size_t t = (size_t)nreg; t < sd.size(); ++t) {
      coop_maxp = std::max<int>(coop_maxp, sd[t].P);
      coop_maxnb = std::max(coop_maxnb, sd[t].nrow + sd[t].ncol);
    }
    size_t best = SIZE_MAX;
    std::vector<CoopLaunch> cand;
    for (int cpt : {1, 2, 4, 8}) {
      const int cap = std::min(1024, sparsify_coop_capacity<T>(cpt, coop_maxp, coop_maxnb));
      cand.clear();
      bool ok = cap > 0;
      for (size_t t = (size_t)nreg; ok && t < sd.size(); ++t) {
        const int nb_t = (sd[t].mmax + 64 * cpt - 1) / (64 * cpt);
        if (nb_t > cap) ok = false;
        else if (cand.empty() || cand.back().blocks + nb_t > cap)
          cand.push_back({(int64_t)t, (int64_t)t + 1, nb_t, kmax_of(sd[t])});
        else {
          cand.back().end = (int64_t)t + 1;
          cand.back().blocks += nb_t;
        }
      }
      if (ok && cand.size() < best) {
        best = cand.size();
        coop = cand;
        coop_cpt = cpt;
      }
    }
    if (coop_cpt > 0) {
      ncoop = (int64_t)sd.size() - nreg;
      for (const CoopLaunch& L : coop) {
        int first = 0;
        for (int64_t t = L.begin; t < L.end; ++t) {
          const int nb_t = (sd[t].mmax + 64 * coop_cpt - 1) / (64 * coop_cpt);
          items.push_back({first, nb_t});
          first += nb_t;
        }
        coop_blocks = std::max(coop_blocks, L.blocks);
      }
    }
  }
  // the rest: interfaces of at most 64 (FP32) or 32 (FP64) unknowns to the LDS
  // kernel, the others to the generic one
  constexpr int kSmallP = sizeof(T) == 4 ? 64 : 32;
  const int64_t nrest0 = nreg + ncoop;
  std::stable_partition(sd.begin() + nrest0, sd.end(), [](const SpDesc<T>& q) { return q.P <= kSmallP; });
  int64_t nsmall = 0;
  int pmax_small = 1, mmax_small = 1;
  for (size_t t = (size_t)nrest0; t < sd.size(); ++t)
    if (sd[t].P <= kSmallP) {
      ++nsmall;
      pmax_small = std::max<int>(pmax_small, sd[t].P);
      mmax_small = std::max<int>(mmax_small, sd[t].mmax);
    }
  const int pclass = pmax_small <= 16 ? 16 : (pmax_small <= 32 ? 32 : 64);
  const size_t cmax_small = (size_t)(pclass + 1) * mmax_small;
  SpDesc<T>* dsd = up.upload(wk, sd, s);
  if (!dnb) dnb = up.upload(wk, nb, s);
  double* ckey = nullptr;
  int* cpos = nullptr;
  T* ccol = nullptr;
  int* done = nullptr;
  CoopItem* ditems = nullptr;
  if (ncoop > 0) {
    // candidate slots are reused launch after launch (stream order); done
    // flags are per launch
    ckey = wk.alloc_n<double>(2 * (size_t)coop_blocks, s);
    cpos = wk.alloc_n<int>(2 * (size_t)coop_blocks, s);
    ccol = wk.alloc_n<T>(2 * (size_t)coop_blocks * coop_maxp, s);
    done = wk.alloc_n<int>(2 * (size_t)ncoop, s);
    ditems = up.upload(wk, items, s);
    launch_zero_ops({{done, 2 * ncoop * (int64_t)sizeof(int)}}, up, wk, s);
  }
  // one profiler record per kernel launch (the work is added after the rank
  // readback)
  for (const auto& g : groups) {
    ProfScope ps("sparsify", s, 0.0, 0.0);
    launch_sparsify_reg<T>(dsd + g[0], g[1] - g[0], dnb, (int)g[2], (int)g[3], max_nb, s);
  }
  for (const CoopLaunch& L : coop) {
    const int64_t i0 = L.begin - nreg, ni = L.end - L.begin;
    ProfScope ps("sparsify", s, 0.0, 0.0);
    if (!launch_sparsify_coop<T>(dsd + L.begin, ditems + i0, (int)ni, L.blocks, coop_cpt, dnb, coop_maxp, coop_maxnb,
                                 ckey, cpos, ccol, done + 2 * i0, L.kmax, s))
      throw Error(SPAQR_EDEVICE, "cooperative CPQR no longer fits the device");
  }
  if (nsmall > 0) {
    ProfScope ps("sparsify", s, 0.0, 0.0);
    launch_sparsify_small<T>(dsd + nrest0, nsmall, dnb, pmax_small, max_nb, cmax_small, s);
  }
  if ((int64_t)sd.size() > nrest0 + nsmall) {
    ProfScope ps("sparsify", s, 0.0, 0.0);
    launch_sparsify<T>(dsd + nrest0 + nsmall, (int64_t)sd.size() - nrest0 - nsmall, dnb, max_pc, max_nb, s);
  }
}

// FP32 interfaces the downdated-norm CPQR takes (as in sparsify_batch).
static bool dd_takes(const SpDesc<float>& q) {
  return q.P >= 1 && q.P <= 64 && q.mmax <= sparsify_dd_capacity(q.P);
}

// Interfaces of consecutive colours gathered for one dataflow launch of the
// downdated-norm CPQR (cpqr_dd = 2).
struct DDSegment {
  std::vector<SpDesc<float>> sd;
  std::vector<SpNbr> nb;
  std::vector<int> colour;
  void add(SpDesc<float> d, const std::vector<SpNbr>& src, int c) {
    const int64_t o = (int64_t)nb.size();
    nb.insert(nb.end(), src.begin() + d.nb, src.begin() + d.nb + d.nrow + d.ncol);
    d.nb = o;
    sd.push_back(d);
    colour.push_back(c);
  }
};

// Launches a segment: a single colour as before; several colours as one
// launch in which an interface waits only for its adjacent interfaces of
// earlier colours (the sequential order of Section 2.6 orders nothing
// else: an interface's sparsification reads and writes only the blocks it
// shares with its neighbours, and the ranks of those neighbours).  Items are
// ordered by colour, then largest first within a colour.
static void flush_dd_segment(DDSegment& g, Stager& up, DevArena& wk, hipStream_t s, int* err) {
  if (g.sd.empty()) return;
  if (g.colour.front() == g.colour.back()) {
    sparsify_batch<float>(g.sd, g.nb, up, wk, s, err);
    g = DDSegment{};
    return;
  }
  const size_t n = g.sd.size();
  std::vector<size_t> ord(n);
  for (size_t t = 0; t < n; ++t) ord[t] = t;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
    if (g.colour[a] != g.colour[b]) return g.colour[a] < g.colour[b];
    return (int64_t)g.sd[a].P * g.sd[a].mmax > (int64_t)g.sd[b].P * g.sd[b].mmax;
  });
  std::vector<SpDesc<float>> sd(n);
  std::vector<int> col(n);
  // an interface is identified by its factorization's size table and cluster
  std::map<std::pair<const int*, int32_t>, int> at;
  for (size_t t = 0; t < n; ++t) {
    sd[t] = g.sd[ord[t]];
    col[t] = g.colour[ord[t]];
    at.emplace(std::make_pair(static_cast<const int*>(sd[t].rank), sd[t].cluster), (int)t);
  }
  std::vector<int> pp(n + 1, 0), pr;
  int max_nb = 0, lc_rows = 0;
  for (size_t t = 0; t < n; ++t) {
    const SpDesc<float>& q = sd[t];
    max_nb = std::max(max_nb, q.nrow + q.ncol);
    lc_rows = std::max(lc_rows, sparsify_dd_lc_rows(q.P, q.mmax));
    const size_t b0 = pr.size();
    for (int b = 0; b < q.nrow + q.ncol; ++b) {
      const auto it = at.find({q.rank, g.nb[q.nb + b].cluster});
      if (it != at.end() && col[it->second] < col[t]) pr.push_back(it->second);
    }
    std::sort(pr.begin() + b0, pr.end());
    pr.erase(std::unique(pr.begin() + b0, pr.end()), pr.end());
    pp[t + 1] = (int)pr.size();
  }
  std::vector<int> succ(n, 0);
  for (int q : pr) succ[q] = 1;
  if (pr.empty()) pr.push_back(0);
  SpDesc<float>* dsd = up.upload(wk, sd, s);
  SpNbr* dnb = up.upload(wk, g.nb, s);
  int* dpp = up.upload(wk, pp, s);
  int* dpr = up.upload(wk, pr, s);
  int* dsu = up.upload(wk, succ, s);
  int* cnt = wk.alloc_n<int>(n + 1, s);
  launch_zero_ops({{cnt, (int64_t)((n + 1) * sizeof(int))}}, up, wk, s);
  const DDFlow fl{cnt, cnt + 1, dpp, dpr, dsu, err};
  {
    ProfScope ps("sparsify", s, 0.0, 0.0);
    launch_sparsify_dd(dsd, (int64_t)n, dnb, max_nb, lc_rows, s, &fl);
  }
  g = DDSegment{};
}

// One stage of every factorization in es, in two halves: stage_launch plans
// and enqueues everything up to the rank readback and records bx.ev;
// stage_finish waits for that event, finishes the stage on the host and
// enqueues the merges.  Between the two the host is free to plan another
// batch whose work then queues behind this one.
template <typename T>
void stage_launch(const std::vector<Engine<T>*>& es, BatchCtx& bx, hipStream_t s) {
  bx.begin();
  bx.pe = std::make_shared<PhaseEvents>();
  bx.pe->record(0, s);
  for (Engine<T>* e : es) e->note_phases(bx.pe);
  Stager& up = bx.st[bx.cur];
  DevArena& wk = bx.work[bx.cur];
  const size_t ne = es.size();
  std::vector<StagePlan<T>> pl(ne);
  // zero fills requested by the plan parts so far, before their launches
  auto flush_zero = [&]() {
    std::vector<ZeroOp> z;
    for (auto& p : pl) {
      append(z, p.zero);
      p.zero.clear();
    }
    launch_zero_ops(z, up, wk, s);
  };
  {
    HostScope hs("host_plan_fronts");
    // a batch of one plans its own fronts on the host threads
    for (size_t e = 0; e < ne; ++e) es[e]->set_host_pool(ne == 1 ? bx.host_pool() : nullptr);
    bx.each(ne, [&](int e) { es[e]->plan_fronts(pl[e]); });
  }
  flush_zero();
  // fronts, colour by colour
  {
  HostScope hs_fronts("host_launch_fronts");
  size_t nc = 0;
  for (auto& p : pl) nc = std::max(nc, p.fronts.size());
  for (size_t c = 0; c < nc; ++c) {
    std::vector<std::pair<int, std::vector<QRDesc<T>>>> qparts;
    double fl = 0.0, by = 0.0;
    for (auto& p : pl) {
      if (c >= p.fronts.size()) continue;
      qparts.emplace_back(p.jbf, p.fronts[c].qr);
      fl += p.fronts[c].flops;
      by += p.fronts[c].bytes;
    }
    std::vector<const std::vector<CopyTile<T>>*> lists;
    for (auto& p : pl)
      if (c < p.fronts.size())
        for (const auto& v : p.fronts[c].gather) lists.push_back(&v);
    copy_concat<T>(bx, up, wk, lists.size(), [&](int i) -> const std::vector<CopyTile<T>>& { return *lists[i]; },
                   false, s, "copy_front_gather");
    {
      HostScope hs("host_launch_qr");
      launch_qr_groups<T>(qparts, "front_qr", fl, by, up, wk, s);
    }
    {
      // trailing slices of split fronts, grouped by (panel width, slice width)
      std::map<std::pair<int, int>, std::pair<int, std::vector<TrailDesc<T>>>> tg;
      double tfl = 0.0, tby = 0.0;
      for (auto& p : pl) {
        if (c >= p.fronts.size() || p.fronts[c].trail.empty()) continue;
        auto& e = tg[{p.jbf, p.fronts[c].trail_cw}];
        e.first = std::max(e.first, p.fronts[c].trail_max_m);
        append(e.second, p.fronts[c].trail);
        for (const TrailDesc<T>& t : p.fronts[c].trail) {
          // V^T C and C - V (T^T W) over the slice: 4 m n cw; C read and written once
          tfl += 4.0 * t.m * (double)t.n * t.cw;
          tby += 2.0 * t.m * (double)t.cw * sizeof(T);
        }
      }
      if (!tg.empty()) {
        ProfScope ps("front_trail", s, tfl, tby);
        for (auto& kv : tg) {
          TrailDesc<T>* d = up.upload(wk, kv.second.second, s);
          launch_trail<T>(d, (int64_t)kv.second.second.size(), kv.first.first, kv.first.second, kv.second.first, s);
        }
      }
      // the matrix-core form: T factors of every 64-reflector block, then
      // the 64-column tiles
      std::vector<WYBlock<T>> wyb;
      std::vector<WYTile<T>> wyt;
      double mfl = 0.0, mby = 0.0;
      for (auto& p : pl) {
        if (c >= p.fronts.size()) continue;
        append(wyb, p.fronts[c].wyb);
        append(wyt, p.fronts[c].wyt);
      }
      for (const WYTile<T>& t : wyt) {
        mfl += 4.0 * t.m * (double)t.n * t.cw;
        mby += 2.0 * t.m * (double)t.cw * sizeof(T);
      }
      if (!wyt.empty()) {
        double gfl = 0.0;
        for (const WYBlock<T>& b : wyb) gfl += 2.0 * (b.m - b.j0) * (double)kWYBlock * kWYBlock;
        WYBlock<T>* db = up.upload(wk, wyb, s);
        {
          ProfScope ps("front_wy_blocks", s, gfl, 0.0);
          launch_wy_tblock<T>(db, (int64_t)wyb.size(), s);
        }
        WYTile<T>* dt = up.upload(wk, wyt, s);
        ProfScope ps("front_trail", s, mfl, mby);
        launch_trail_mfma<T>(dt, (int64_t)wyt.size(), s);
      }
    }
    {
      std::vector<const std::vector<CopyTile<T>>*> sl;
      for (auto& p : pl)
        if (c < p.fronts.size())
          for (const auto& v : p.fronts[c].scatter) sl.push_back(&v);
      copy_concat<T>(bx, up, wk, sl.size(), [&](int i) -> const std::vector<CopyTile<T>>& { return *sl[i]; }, false,
                     s, "copy_front_scatter");
    }
  }
  copy_concat<T>(bx, up, wk, ne, [&](int e) -> const std::vector<CopyTile<T>>& { return pl[e].pack; }, true, s,
                 "copy_front_pack");
  }
  bx.pe->record(1, s);
  // block-diagonal scaling
  {
    HostScope hs("host_plan_scale");
    bx.each(ne, [&](int e) { es[e]->plan_scale(pl[e]); });
  }
  flush_zero();
  {
    HostScope hs("host_launch_scale");
    std::vector<CopyTile<T>> g, pk;
    std::vector<std::pair<int, std::vector<QRDesc<T>>>> qparts;
    std::vector<ScaleFac<T>> fac;
    struct SGroup {
      int max_p = 1, max_rows = 1, max_cols = 1;
      std::vector<ScaleBlk<T>> blk;
      // blocks of at most 16, 32 and 64 rows and columns: one launch per
      // class so that small blocks do not pay LDS sized for the largest
      int small_rows[3] = {1, 1, 1}, small_cols[3] = {1, 1, 1};
      std::vector<ScaleBlk<T>> small[3];
    };
    std::map<int, SGroup> sgroups;  // by panel width; blocks of at most 64 x 64 apart
    double qfl = 0.0, qby = 0.0, sfl = 0.0, sby = 0.0;
    for (auto& p : pl) {
      append(g, p.sgather);
      append(pk, p.spack);
      qparts.emplace_back(p.jbs, p.sqr);
      for (const QRDesc<T>& q : p.sqr) {
        qfl += 4.0 / 3.0 * (double)q.n * q.n * q.n;
        qby += 2.0 * (double)q.n * q.n * sizeof(T);
      }
      const int base = (int)fac.size();
      append(fac, p.fac);
      SGroup& sg = sgroups[p.jbs];
      sg.max_p = std::max(sg.max_p, p.max_p);
      for (ScaleBlk<T> b : p.sblk) {
        if (b.fi >= 0) b.fi += base;
        if (b.fj >= 0) b.fj += base;
        if (b.rows <= tuning().scale_small && b.cols <= tuning().scale_small) {
          const int e = std::max(b.rows, b.cols), cl = e <= 16 ? 0 : (e <= 32 ? 1 : 2);
          sg.small_rows[cl] = std::max(sg.small_rows[cl], b.rows);
          sg.small_cols[cl] = std::max(sg.small_cols[cl], b.cols);
          sg.small[cl].push_back(b);
        } else {
          sg.max_rows = std::max(sg.max_rows, b.rows);
          sg.max_cols = std::max(sg.max_cols, b.cols);
          sg.blk.push_back(b);
        }
        sfl += 4.0 * b.rows * b.rows * (double)b.cols + (double)b.rows * b.cols * b.cols;
        sby += 2.0 * b.rows * (double)b.cols * sizeof(T);
      }
    }
    copy_batch(g, false, up, wk, s, "copy_scale_gather");
    launch_qr_groups<T>(qparts, "scale_qr", qfl, qby, up, wk, s);
    copy_batch(pk, true, up, wk, s, "copy_scale_pack");
    if (!fac.empty()) {
      ScaleFac<T>* dfac = up.upload(wk, fac, s);
      ProfScope ps("scale_blocks", s, sfl, sby);
      for (auto& kv : sgroups) {
        const SGroup& g = kv.second;
        for (int cl = 0; cl < 3; ++cl)
          if (!g.small[cl].empty()) {
            ScaleBlk<T>* dsb = up.upload(wk, g.small[cl], s);
            launch_scale_small<T>(dsb, (int64_t)g.small[cl].size(), dfac, kv.first, g.small_rows[cl],
                                  g.small_cols[cl], s);
          }
        if (g.blk.empty()) continue;
        const int cw = kv.first >= 4 ? trail_width(g.max_rows, sizeof(T)) : 0;
        if (cw == 0) {
          ScaleBlk<T>* dsb = up.upload(wk, g.blk, s);
          launch_scale<T>(dsb, (int64_t)g.blk.size(), dfac, kv.first, g.max_p, g.max_rows, g.max_cols, s);
          continue;
        }
        // larger blocks: Q_i^T by 16-column slices (the trailing-update
        // kernel reading V row-major from the scaling QR's workspace), the
        // diagonal blocks set to I, then B R_j^{-1}
        std::vector<ScaleBlk<T>> ident, rest;
        std::vector<TrailDesc<T>> left;
        // on the matrix cores: T factors per interface (once, whatever the
        // number of its blocks), then 64-column tiles of every block
        const bool mfma = tuning().trail_mfma != 0;
        std::map<int, int64_t> tb_of;  // interface -> offset of its T blocks
        std::vector<WYBlock<T>> wyb;
        std::vector<WYTile<T>> wyt;
        std::vector<int64_t> wyt_off;  // offset of each tile's T blocks
        int64_t tb_tot = 0;
        int lm = 1;
        for (const ScaleBlk<T>& b : g.blk) {
          if (b.fi >= 0 && b.fi == b.fj) {
            ident.push_back(b);
            continue;
          }
          rest.push_back(b);
          if (b.fi < 0) continue;
          const ScaleFac<T>& f = fac[b.fi];
          lm = std::max(lm, b.rows);
          if (mfma) {
            auto it = tb_of.find(b.fi);
            if (it == tb_of.end()) {
              it = tb_of.emplace(b.fi, tb_tot).first;
              tb_tot += (int64_t)(f.P + kWYBlock - 1) / kWYBlock * kWYBlock * kWYBlock;
            }
            for (int c0 = 0; c0 < b.cols; c0 += kWYBlock) {
              wyt.push_back({f.vw, nullptr, b.B, f.flag, b.rows, b.rows, f.ldw, c0, std::min(kWYBlock, b.cols - c0),
                             b.cols});
              wyt_off.push_back(it->second);
            }
            continue;
          }
          for (int c0 = 0; c0 < b.cols; c0 += cw)
            left.push_back({f.vw, f.tpan, b.B, f.flag, b.rows, b.rows, f.ldw, c0, std::min(cw, b.cols - c0), b.cols});
        }
        if (!left.empty()) {
          TrailDesc<T>* dl = up.upload(wk, left, s);
          launch_trail<T>(dl, (int64_t)left.size(), kv.first, cw, lm, s);
        }
        if (!wyt.empty()) {
          T* tb = wk.alloc_n<T>((size_t)tb_tot, s);
          for (const auto& kvf : tb_of) {
            const ScaleFac<T>& f = fac[kvf.first];
            for (int j0 = 0; j0 < f.P; j0 += kWYBlock)
              wyb.push_back({f.vw, f.tau, tb + kvf.second + (int64_t)(j0 / kWYBlock) * kWYBlock * kWYBlock, f.P, f.P,
                             f.ldw, j0});
          }
          for (size_t q = 0; q < wyt.size(); ++q) wyt[q].tblk = tb + wyt_off[q];
          WYBlock<T>* db = up.upload(wk, wyb, s);
          launch_wy_tblock<T>(db, (int64_t)wyb.size(), s);
          WYTile<T>* dt = up.upload(wk, wyt, s);
          launch_trail_mfma<T>(dt, (int64_t)wyt.size(), s);
        }
        if (!ident.empty()) {
          ScaleBlk<T>* di = up.upload(wk, ident, s);
          launch_scale_small<T>(di, (int64_t)ident.size(), dfac, kv.first, 1, 1, s);  // identity fill only
        }
        if (!rest.empty()) {
          ScaleBlk<T>* dr = up.upload(wk, rest, s);
          launch_scale_right<T>(dr, (int64_t)rest.size(), dfac, g.max_rows, s);
        }
      }
    }
  }
  bx.pe->record(2, s);
  // sparsification, colour by colour; team_err: set by a team CPQR whose
  // barrier wait ran out or a dataflow CPQR whose dependency wait ran out
  // (read back with the ranks, thrown in stage_finish)
  int* team_err = wk.alloc_n<int>(1, s);
  launch_zero_ops({{team_err, (int64_t)sizeof(int)}}, up, wk, s);
  {
    HostScope hs("host_plan_sparsify");
    bx.each(ne, [&](int e) { es[e]->plan_sparsify(pl[e]); });
  }
  flush_zero();
  {
  HostScope hs_sp("host_launch_sparsify");
  size_t nsc = 0;
  for (auto& p : pl) nsc = std::max(nsc, p.sp.size());
  // cpqr_dd = 2: the FP32 interfaces the downdated-norm CPQR takes are
  // gathered over consecutive colours of fewer such interfaces than the
  // device has CUs (where one launch per colour leaves most of them idle)
  // into one dataflow launch, cut before a colour's other interfaces or a
  // larger colour launch; larger colours keep one launch each, whose host
  // planning overlaps the previous launch
  constexpr int kDDFlowMaxColour = 256;
  DDSegment seg;
  for (size_t c = 0; c < nsc; ++c) {
    std::vector<SpDesc<T>> sd;
    std::vector<SpNbr> nb;
    for (auto& p : pl) {
      if (c >= p.sp.size()) continue;
      const int64_t base = (int64_t)nb.size();
      append(nb, p.sp[c].nb);
      for (SpDesc<T> d : p.sp[c].sd) {
        d.nb += base;
        sd.push_back(d);
      }
    }
    if constexpr (std::is_same<T, float>::value) {
      int ndd = 0;
      for (const SpDesc<T>& d : sd) ndd += dd_takes(d) ? 1 : 0;
      if (tuning().cpqr_dd == 2 && ndd < kDDFlowMaxColour) {
        std::vector<SpDesc<T>> rest;
        for (const SpDesc<T>& d : sd) {
          if (dd_takes(d)) seg.add(d, nb, (int)c);
          else rest.push_back(d);
        }
        if (!rest.empty()) {
          flush_dd_segment(seg, up, wk, s, team_err);
          sparsify_batch<T>(rest, nb, up, wk, s, team_err);
        }
        continue;
      }
      flush_dd_segment(seg, up, wk, s, team_err);
    }
    sparsify_batch<T>(sd, nb, up, wk, s, team_err);
  }
  if constexpr (std::is_same<T, float>::value) flush_dd_segment(seg, up, wk, s, team_err);
  size_t nsu = 0;
  for (auto& p : pl) nsu = std::max(nsu, p.spu.size());
  for (size_t c = 0; c < nsu; ++c) {
    std::vector<SpuDesc<T>> sd;
    std::vector<SpNbr> nb;
    for (auto& p : pl) {
      if (c >= p.spu.size()) continue;
      const int64_t base = (int64_t)nb.size();
      append(nb, p.spu[c].nb);
      for (SpuDesc<T> d : p.spu[c].sd) {
        d.nb += base;
        sd.push_back(d);
      }
    }
    if (sd.empty()) continue;
    int max_p = 0;
    for (const SpuDesc<T>& d : sd) max_p = std::max(max_p, (int)d.P);
    SpuDesc<T>* dsd = up.upload(wk, sd, s);
    SpNbr* dnb = up.upload(wk, nb, s);
    ProfScope ps("sparsify_unscaled", s, 0.0, 0.0);
    launch_sparsify_unscaled<T>(dsd, dnb, (int64_t)sd.size(), max_p, s);
  }
  {
    // dense interface operators, one launch per size class (16, 32, 64)
    std::vector<ApIface<T>> form[3];
    for (auto& p : pl)
      for (const ApIface<T>& q : p.form) form[q.P <= 16 ? 0 : (q.P <= 32 ? 1 : 2)].push_back(q);
    for (int cl = 0; cl < 3; ++cl)
      if (!form[cl].empty()) {
        ApIface<T>* d = up.upload(wk, form[cl], s);
        double by = 0.0;  // reflectors read, both operators written
        for (const ApIface<T>& q : form[cl]) by += 4.0 * q.P * (double)q.P * sizeof(T);
        ProfScope ps("iface_form", s, 0.0, by);
        launch_iface_form<T>(d, (int64_t)form[cl].size(), 16 << cl, s);
      }
  }
  }
  bx.pe->record(3, s);
  // ranks and flags of every factorization: one gather, one copy back
  {
    std::vector<IntCopy> ops;
    std::vector<int32_t> base(es.size());
    int32_t tot = 0;
    for (size_t i = 0; i < es.size(); ++i) {
      base[i] = tot;
      es[i]->readback_ops(ops, tot);
      tot += es[i]->readback_ints();
    }
    ops.push_back({team_err, tot, 1});
    bx.team_err_at = tot++;
    int32_t* d = wk.alloc_n<int32_t>((size_t)tot, s);
    launch_gather_ints(ops.data(), (int)ops.size(), d, s);
    if (bx.rb.size < (size_t)tot * sizeof(int32_t)) {
      pinned_release(bx.rb);
      bx.rb = pinned_acquire((size_t)tot * sizeof(int32_t));
    }
    int32_t* h = reinterpret_cast<int32_t*>(bx.rb.p);
    SPAQR_HIP(hipMemcpyAsync(h, d, (size_t)tot * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    for (size_t i = 0; i < es.size(); ++i) es[i]->readback_to(h + base[i]);
  }
  if (!bx.ev) SPAQR_HIP(hipEventCreateWithFlags(&bx.ev, hipEventDisableTiming));
  SPAQR_HIP(hipEventRecord(bx.ev, s));
}

template <typename T>
void stage_finish(const std::vector<Engine<T>*>& es, BatchCtx& bx, hipStream_t s) {
  Stager& up = bx.st[bx.cur];
  DevArena& wk = bx.work[bx.cur];
  const size_t ne = es.size();
  {
    HostScope hs("host_wait_gpu");
    SPAQR_HIP(hipEventSynchronize(bx.ev));
  }
  if (bx.team_err_at >= 0 && reinterpret_cast<const int32_t*>(bx.rb.p)[bx.team_err_at] != 0)
    throw Error(SPAQR_EDEVICE, "a CPQR team barrier or dependency wait ran out (results of the stage invalid)");
  std::vector<MergePlan<T>> mp(ne);
  {
    HostScope hs("host_finish");
    for (size_t e = 0; e < ne; ++e) es[e]->set_host_pool(ne == 1 ? bx.host_pool() : nullptr);
    bx.each(ne, [&](int e) { es[e]->finish(mp[e]); });
  }
  HostScope hs_merge("host_launch_merge");
  std::vector<ZeroOp> z;
  for (auto& m : mp) append(z, m.zero);
  launch_zero_ops(z, up, wk, s);
  std::vector<const std::vector<CopyTile<T>>*> lists;
  for (auto& m : mp)
    for (const auto& v : m.tiles) lists.push_back(&v);
  copy_concat<T>(bx, up, wk, lists.size(), [&](int i) -> const std::vector<CopyTile<T>>& { return *lists[i]; }, false,
                 s, "copy_merge");
  if (bx.pe) bx.pe->record(4, s);
  bx.pe.reset();
}

template <typename T>
void run_stage_batch(const std::vector<Engine<T>*>& es, BatchCtx& bx, hipStream_t s) {
  stage_launch<T>(es, bx, s);
  stage_finish<T>(es, bx, s);
}

template <typename T>
void Engine<T>::apply_dev(const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs) {
  const size_t need = (size_t)S_.n * nrhs;
  if (apply_ws_cap_ < need) {
    drop_graphs();
    dev_free(apply_ws_, s_);
    apply_ws_ = static_cast<double*>(dev_alloc(need * sizeof(double), s_));
    apply_ws_cap_ = need;
  }
  const int64_t N = S_.n;
  launch_gather_perm(apply_ws_, b, ldb, d_perm_, N, nrhs, s_);
  // the sweeps, the same launches at every apply of a given width: replayed
  // from a HIP graph captured at the second apply of that width (the first
  // runs eagerly, which also sets every kernel's LDS attribute); eager while
  // the profiler times launches
  if (prof_on()) {
    sweeps(apply_ws_, nrhs);
  } else {
    auto it = graphs_.find(nrhs);
    if (it == graphs_.end()) {
      sweeps(apply_ws_, nrhs);
      graphs_[nrhs] = nullptr;
    } else {
      if (!it->second) it->second = capture_sweeps(apply_ws_, nrhs);
      SPAQR_HIP(hipGraphLaunch(it->second, s_));
    }
  }
  launch_scatter_perm(x, ldx, apply_ws_, d_perm_, d_dc_, N, nrhs, s_);
  SPAQR_HIP(hipGetLastError());
}

template <typename T>
hipGraphExec_t Engine<T>::capture_sweeps(double* xh, int nrhs) {
  return capture_graph([&](hipStream_t cs) { sweeps(xh, nrhs, cs); });
}

template <typename T>
void Engine<T>::drop_graphs() {
  if (graphs_.empty()) return;
  (void)hipStreamSynchronize(s_);
  for (auto& kv : graphs_)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  graphs_.clear();
}

template <typename T>
void Engine<T>::apply_ws(const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs, double* xh) {
  const int64_t N = S_.n;
  launch_gather_perm(xh, b, ldb, d_perm_, N, nrhs, s_);
  sweeps(xh, nrhs);
  launch_scatter_perm(x, ldx, xh, d_perm_, d_dc_, N, nrhs, s_);
  SPAQR_HIP(hipGetLastError());
}

// The forward sweep (Q^T, stage L .. 1) and the backward sweep (W^{-1},
// stage 1 .. L) on the permuted vectors xh (N x nrhs, in place).
template <typename T>
void Engine<T>::sweeps(double* xh, int nrhs, hipStream_t s) {
  const int64_t N = S_.n;
  const int L = S_.L;
  for (int k = L; k >= 1; --k) {
    const StageApply<T>& a = ap_[k];
    for (size_t c = 0; c + 1 < a.colour_ptr.size(); ++c) {
      const int64_t cnt = a.colour_ptr[c + 1] - a.colour_ptr[c];
      if (cnt == 0) continue;
      ProfScope ps("apply_front_fwd", s, a.fwd_flops[c] * nrhs, a.fwd_fac_bytes[c] + a.fwd_vec_bytes[c] * nrhs);
      launch_front_fwd_wy<T>(a.fronts + a.colour_ptr[c], cnt, a.jb, a.colour_max_m[c], xh, N, nrhs, s);
    }
    if (a.nifaces) {
      ProfScope ps("apply_iface_fwd", s, a.if_fwd_flops * nrhs, a.if_fwd_fac_bytes + a.if_vec_bytes * nrhs);
      launch_iface_dense<T>(a.ifaces, a.nifaces_small, false, xh, N, nrhs, s, a.dense_max_p);
      launch_iface_fwd<T>(a.ifaces + a.nifaces_small, a.nifaces - a.nifaces_small, a.max_p, xh, N, nrhs, s);
    }
  }
  for (int k = 1; k <= L; ++k) {
    const StageApply<T>& a = ap_[k];
    if (a.nifaces) {
      ProfScope ps("apply_iface_bwd", s, a.if_bwd_flops * nrhs, a.if_bwd_fac_bytes + a.if_vec_bytes * nrhs);
      launch_iface_dense<T>(a.ifaces, a.nifaces_small, true, xh, N, nrhs, s, a.dense_max_p);
      launch_iface_bwd<T>(a.ifaces + a.nifaces_small, a.nifaces - a.nifaces_small, a.max_p, xh, N, nrhs, s);
    }
    if (a.nfronts) {
      ProfScope ps("apply_front_bwd", s, a.bwd_flops * nrhs, a.bwd_fac_bytes + a.bwd_vec_bytes * nrhs);
      launch_front_bwd_reg<T>(a.fronts, a.nfronts, a.max_n, a.max_k, xh, N, nrhs, s);
    }
  }
}

// ------------------------------------------------- apply across problems
// The preconditioners of several factorizations, each applied to its own
// columns, with one launch per phase of the apply: the descriptors of every
// problem's stage k (colour c) are concatenated, each carrying the offset of
// its problem's permuted vector in one shared buffer, so an apply costs the
// launches of the deepest problem alone.
template <typename T>
class BatchApply {
 public:
  // cols[i]: the columns of problem i (indices into the caller's b and x)
  BatchApply(const std::vector<Engine<T>*>& es, const std::vector<std::vector<int>>& cols, hipStream_t s)
      : s_(s) {
    const size_t ne = es.size();
    std::vector<int64_t> off(ne, 0);
    int R = 1, L = 0;
    for (size_t i = 0; i < ne; ++i) {
      off[i] = Ntot_;
      Ntot_ += es[i]->n();
      R = std::max<int>(R, (int)cols[i].size());
      L = std::max(L, es[i]->levels());
      max_n_ = std::max(max_n_, es[i]->n());
    }
    SPAQR_REQUIRE(Ntot_ < (int64_t(1) << 31), SPAQR_EINVAL, "batched apply: too many unknowns in one batch");
    R_ = R;
    std::vector<PermCol> pc;
    for (size_t i = 0; i < ne; ++i)
      for (size_t r = 0; r < cols[i].size(); ++r)
        pc.push_back({cols[i][r], off[i] + (int64_t)r * Ntot_, es[i]->perm_dev(), es[i]->colscale_dev(), es[i]->n()});
    ncols_ = (int)pc.size();
    lv_.assign(L + 1, Level());
    // every descriptor list goes up in one staged copy: packed here, the
    // device pointers set once the region is known
    std::vector<char> pack;
    std::vector<std::function<void(char*)>> fix;
    auto put = [&pack](const void* p, size_t bytes) {
      const size_t o = (pack.size() + 255) / 256 * 256;
      pack.resize(o + bytes);
      std::memcpy(pack.data() + o, p, bytes);
      return o;
    };
    for (int k = 1; k <= L; ++k) {
      Level& v = lv_[k];
      std::map<int, std::vector<ApFront<T>>> fwd_by_c_jb;  // key: colour * 64 + jb
      std::map<int, int> fwd_max_m;
      std::vector<ApFront<T>> bwd;
      std::vector<ApIface<T>> dense, other;
      for (size_t i = 0; i < ne; ++i) {
        if (k > es[i]->levels()) continue;
        const StageApply<T>& a = es[i]->stage_apply()[k];
        for (size_t c = 0; c + 1 < a.colour_ptr.size(); ++c)
          for (int64_t t = a.colour_ptr[c]; t < a.colour_ptr[c + 1]; ++t) {
            ApFront<T> d = a.h_fronts[t];
            d.xoff = (int32_t)off[i];
            const int key = (int)c * 64 + a.jb;
            fwd_by_c_jb[key].push_back(d);
            int& mm = fwd_max_m[key];
            mm = std::max(mm, a.colour_max_m[c]);
          }
        for (ApFront<T> d : a.h_fronts) {
          d.xoff = (int32_t)off[i];
          bwd.push_back(d);
        }
        v.max_n = std::max(v.max_n, a.max_n);
        v.max_k = std::max(v.max_k, a.max_k);
        for (int64_t t = 0; t < (int64_t)a.h_ifaces.size(); ++t) {
          ApIface<T> d = a.h_ifaces[t];
          d.xoff = (int32_t)off[i];
          (t < a.nifaces_small ? dense : other).push_back(d);
          if (t < a.nifaces_small) v.dense_max_p = std::max(v.dense_max_p, (int)d.P);
        }
        v.max_p = std::max(v.max_p, a.max_p);
        for (size_t c = 0; c < a.fwd_flops.size(); ++c) {
          v.fwd_flops += a.fwd_flops[c];
          v.fwd_fac_bytes += a.fwd_fac_bytes[c];
          v.fwd_vec_bytes += a.fwd_vec_bytes[c];
        }
        v.bwd_flops += a.bwd_flops;
        v.bwd_fac_bytes += a.bwd_fac_bytes;
        v.bwd_vec_bytes += a.bwd_vec_bytes;
        v.if_fwd_flops += a.if_fwd_flops;
        v.if_bwd_flops += a.if_bwd_flops;
        v.if_fwd_fac_bytes += a.if_fwd_fac_bytes;
        v.if_bwd_fac_bytes += a.if_bwd_fac_bytes;
        v.if_vec_bytes += a.if_vec_bytes;
      }
      for (auto& kv : fwd_by_c_jb) {
        const size_t o = put(kv.second.data(), kv.second.size() * sizeof(ApFront<T>));
        const size_t i = v.fwd.size();
        v.fwd.push_back({nullptr, (int64_t)kv.second.size(), kv.first % 64, fwd_max_m[kv.first]});
        fix.push_back([&v, i, o](char* b) { v.fwd[i].d = reinterpret_cast<const ApFront<T>*>(b + o); });
      }
      v.nbwd = (int64_t)bwd.size();
      if (!bwd.empty()) {
        const size_t o = put(bwd.data(), bwd.size() * sizeof(ApFront<T>));
        fix.push_back([&v, o](char* b) { v.bwd = reinterpret_cast<const ApFront<T>*>(b + o); });
      }
      v.nif_dense = (int64_t)dense.size();
      v.nif = v.nif_dense + (int64_t)other.size();
      dense.insert(dense.end(), other.begin(), other.end());
      if (!dense.empty()) {
        const size_t o = put(dense.data(), dense.size() * sizeof(ApIface<T>));
        fix.push_back([&v, o](char* b) { v.ifs = reinterpret_cast<const ApIface<T>*>(b + o); });
      }
    }
    if (!pc.empty()) {
      const size_t o = put(pc.data(), pc.size() * sizeof(PermCol));
      fix.push_back([this, o](char* b) { pc_ = reinterpret_cast<const PermCol*>(b + o); });
    }
    if (!pack.empty()) {
      const Stager::Region r = st_.stage(ar_, pack.size(), s_);
      std::memcpy(r.host, pack.data(), pack.size());
      st_.send(r, s_);
      for (auto& f : fix) f(static_cast<char*>(r.dev));
    }
    X_ = ar_.alloc_n<double>((size_t)Ntot_ * R_, s_);
    SPAQR_HIP(hipMemsetAsync(X_, 0, (size_t)Ntot_ * R_ * sizeof(double), s_));
    // (the staging region is released only after the destructor's sync)
  }
  ~BatchApply() {
    (void)hipStreamSynchronize(s_);
    if (gx_) (void)hipGraphExecDestroy(gx_);
  }

  // x[:, cols] = M^{-1} b[:, cols] for this batch's columns; from the second
  // apply on, the sweeps replay a HIP graph captured then (eager while the
  // profiler times launches)
  void apply(const double* b, int64_t ldb, double* x, int64_t ldx) {
    launch_gather_cols(X_, b, ldb, pc_, ncols_, max_n_, s_);
    if (prof_on() || calls_++ == 0) {
      sweeps(s_);
    } else {
      if (!gx_) gx_ = capture_graph([&](hipStream_t cs) { sweeps(cs); });
      SPAQR_HIP(hipGraphLaunch(gx_, s_));
    }
    launch_scatter_cols(x, ldx, X_, pc_, ncols_, max_n_, s_);
    SPAQR_HIP(hipGetLastError());
  }

 private:
  // both sweeps over the batch's permuted vectors X_
  void sweeps(hipStream_t s) {
    const int L = (int)lv_.size() - 1;
    const int nr = R_;
    for (int k = L; k >= 1; --k) {
      const Level& v = lv_[k];
      if (!v.fwd.empty()) {
        ProfScope ps("apply_front_fwd", s, v.fwd_flops * nr, v.fwd_fac_bytes + v.fwd_vec_bytes * nr);
        for (const FwdLaunch& f : v.fwd) launch_front_fwd_wy<T>(f.d, f.n, f.jb, f.max_m, X_, Ntot_, nr, s);
      }
      if (v.nif) {
        ProfScope ps("apply_iface_fwd", s, v.if_fwd_flops * nr, v.if_fwd_fac_bytes + v.if_vec_bytes * nr);
        launch_iface_dense<T>(v.ifs, v.nif_dense, false, X_, Ntot_, nr, s, v.dense_max_p);
        launch_iface_fwd<T>(v.ifs + v.nif_dense, v.nif - v.nif_dense, v.max_p, X_, Ntot_, nr, s);
      }
    }
    for (int k = 1; k <= L; ++k) {
      const Level& v = lv_[k];
      if (v.nif) {
        ProfScope ps("apply_iface_bwd", s, v.if_bwd_flops * nr, v.if_bwd_fac_bytes + v.if_vec_bytes * nr);
        launch_iface_dense<T>(v.ifs, v.nif_dense, true, X_, Ntot_, nr, s, v.dense_max_p);
        launch_iface_bwd<T>(v.ifs + v.nif_dense, v.nif - v.nif_dense, v.max_p, X_, Ntot_, nr, s);
      }
      if (v.nbwd) {
        ProfScope ps("apply_front_bwd", s, v.bwd_flops * nr, v.bwd_fac_bytes + v.bwd_vec_bytes * nr);
        launch_front_bwd_reg<T>(v.bwd, v.nbwd, v.max_n, v.max_k, X_, Ntot_, nr, s);
      }
    }
  }

  struct FwdLaunch {
    const ApFront<T>* d;
    int64_t n;
    int jb, max_m;
  };
  struct Level {
    std::vector<FwdLaunch> fwd;  // colour by colour, one launch per panel width
    const ApFront<T>* bwd = nullptr;
    int64_t nbwd = 0;
    int max_n = 0, max_k = 0;
    const ApIface<T>* ifs = nullptr;  // dense-operator interfaces first
    int64_t nif = 0, nif_dense = 0;
    int max_p = 0, dense_max_p = 0;
    double fwd_flops = 0, fwd_fac_bytes = 0, fwd_vec_bytes = 0, bwd_flops = 0, bwd_fac_bytes = 0, bwd_vec_bytes = 0;
    double if_fwd_flops = 0, if_bwd_flops = 0, if_fwd_fac_bytes = 0, if_bwd_fac_bytes = 0, if_vec_bytes = 0;
  };
  hipStream_t s_;
  DevArena ar_{size_t(8) << 20};
  Stager st_;
  std::vector<Level> lv_;
  const PermCol* pc_ = nullptr;
  double* X_ = nullptr;
  int64_t Ntot_ = 0, max_n_ = 0;
  int R_ = 1, ncols_ = 0;
  int calls_ = 0;
  hipGraphExec_t gx_ = nullptr;
};

// FGMRES operator over the columns of several problems (FP32 and FP64
// factorizations in separate batched applies, one SpMV launch for all).
class MultiOp final : public KrylovOp {
 public:
  MultiOp(const std::vector<EngineBase*>& es, const std::vector<int>& nrhs) {
    SPAQR_REQUIRE(!es.empty() && es.size() == nrhs.size(), SPAQR_EINVAL, "batched solve: bad problem list");
    s_ = es[0]->stream();
    std::vector<Engine<float>*> e32;
    std::vector<Engine<double>*> e64;
    std::vector<std::vector<int>> c32, c64;
    std::vector<SpmvCol> sc;
    int col = 0;
    for (size_t i = 0; i < es.size(); ++i) {
      EngineBase* e = es[i];
      SPAQR_REQUIRE(e->stream() == s_, SPAQR_EINVAL, "batched problems must share one stream");
      SPAQR_REQUIRE(e->stages_left() == 0 && e->error() == SPAQR_OK, SPAQR_EINVAL,
                    "batched solve of an incomplete factorization");
      SPAQR_REQUIRE(nrhs[i] >= 1, SPAQR_EINVAL, "batched solve: a problem without right-hand sides");
      std::vector<int> cs;
      for (int r = 0; r < nrhs[i]; ++r) cs.push_back(col++);
      n_ = std::max(n_, e->n());
      if (e->precision() == 32) {
        auto* ef = static_cast<Engine<float>*>(e);
        e32.push_back(ef);
        c32.push_back(cs);
        for (int r = 0; r < nrhs[i]; ++r) sc.push_back(ef->spmv_col());
      } else {
        auto* ed = static_cast<Engine<double>*>(e);
        e64.push_back(ed);
        c64.push_back(cs);
        for (int r = 0; r < nrhs[i]; ++r) sc.push_back(ed->spmv_col());
      }
    }
    ncols_ = col;
    if (!e32.empty()) b32_.reset(new BatchApply<float>(e32, c32, s_));
    if (!e64.empty()) b64_.reset(new BatchApply<double>(e64, c64, s_));
    sc_ = st_.upload(ar_, sc, s_);
    SPAQR_HIP(hipStreamSynchronize(s_));
  }
  ~MultiOp() override { (void)hipStreamSynchronize(s_); }
  void apply_dev(const double* b, int64_t ldb, double* x, int64_t ldx, int ncols) override {
    SPAQR_REQUIRE(ncols == ncols_, SPAQR_EINVAL, "batched apply: column count differs from the batch");
    if (b32_) b32_->apply(b, ldb, x, ldx);
    if (b64_) b64_->apply(b, ldb, x, ldx);
  }
  void spmv_dev(const double* x, int64_t ldx, double* y, int64_t ldy, int ncols) override {
    SPAQR_REQUIRE(ncols == ncols_, SPAQR_EINVAL, "batched SpMV: column count differs from the batch");
    launch_spmv_cols(sc_, ncols_, n_, x, ldx, y, ldy, s_);
  }
  hipStream_t stream() const override { return s_; }
  int64_t n() const override { return n_; }

 private:
  hipStream_t s_ = nullptr;
  int64_t n_ = 0;
  int ncols_ = 0;
  std::unique_ptr<BatchApply<float>> b32_;
  std::unique_ptr<BatchApply<double>> b64_;
  DevArena ar_{size_t(1) << 20};
  Stager st_;
  const SpmvCol* sc_ = nullptr;
};

}  // namespace

template <typename T>
static void factor_all(Engine<T>* e) {
  BatchCtx bx;
  const std::vector<Engine<T>*> one{e};
  try {
    while (e->stages_left() > 0) run_stage_batch<T>(one, bx, e->stream());
  } catch (...) {
    (void)hipStreamSynchronize(e->stream());
    throw;
  }
  SPAQR_HIP(hipStreamSynchronize(e->stream()));
  if (e->error() != SPAQR_OK) throw Error(e->error(), e->error_message());
}

std::unique_ptr<EngineBase> make_engine_deferred(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S,
                                                 const spaqr_opts& o, hipStream_t stream) {
  SPAQR_REQUIRE(o.eps >= 0.0 && std::isfinite(o.eps), SPAQR_EINVAL, "eps must be finite and >= 0");
  SPAQR_REQUIRE(o.scale == 0 || o.scale == 1, SPAQR_EINVAL, "scale is 0 or 1");
  SPAQR_REQUIRE(o.precision == 32 || o.precision == 64, SPAQR_EINVAL, "precision must be 32 or 64");
  if (o.precision == 32) return std::unique_ptr<EngineBase>(new Engine<float>(A, Ad, S, o, stream));
  return std::unique_ptr<EngineBase>(new Engine<double>(A, Ad, S, o, stream));
}

std::unique_ptr<EngineBase> make_engine(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S,
                                        const spaqr_opts& o, hipStream_t stream) {
  std::unique_ptr<EngineBase> e = make_engine_deferred(A, Ad, S, o, stream);
  if (o.precision == 32) factor_all(static_cast<Engine<float>*>(e.get()));
  else factor_all(static_cast<Engine<double>*>(e.get()));
  return e;
}

// One stage of every factorization in es (each at its own next stage), the
// FP32 and FP64 ones in separate launches.  All must use stream s.
struct BatchDriver {
  BatchCtx b32, b64;
};

BatchDriver* batch_driver_new() { return new BatchDriver(); }
void batch_driver_free(BatchDriver* d) { delete d; }

std::unique_ptr<KrylovOp> make_batch_op(const std::vector<EngineBase*>& es, const std::vector<int>& nrhs) {
  return std::unique_ptr<KrylovOp>(new MultiOp(es, nrhs));
}

static void split_precision(const std::vector<EngineBase*>& es, hipStream_t s, std::vector<Engine<float>*>& f32,
                            std::vector<Engine<double>*>& f64) {
  for (EngineBase* e : es) {
    if (e->stages_left() <= 0) continue;
    SPAQR_REQUIRE(e->stream() == s, SPAQR_EINVAL, "batched factorizations must share one stream");
    if (e->precision() == 32) f32.push_back(static_cast<Engine<float>*>(e));
    else f64.push_back(static_cast<Engine<double>*>(e));
  }
}

void factor_stage_batch(BatchDriver& drv, const std::vector<EngineBase*>& es, hipStream_t s) {
  std::vector<Engine<float>*> f32;
  std::vector<Engine<double>*> f64;
  split_precision(es, s, f32, f64);
  if (!f32.empty()) run_stage_batch<float>(f32, drv.b32, s);
  if (!f64.empty()) run_stage_batch<double>(f64, drv.b64, s);
}


}  // namespace spaqr
