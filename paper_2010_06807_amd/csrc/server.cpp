// Continuous-batching request loop.  Requests (matrix, ordering, options and
// right-hand sides) are copied at submission and queued.  Every step:
//   1. admits queued requests in arrival order while their estimated device
//      memory fits the budget (symbolic analysis and matrix upload happen
//      here, the admitted requests in parallel host threads);
//   2. advances every admitted, still factoring request by one stage in one
//      batched pass: their fronts, scalings and sparsifications share one
//      launch per phase, whatever stage each request is at, so a request that
//      arrives while others are half-way joins the running batch;
//   3. solves the requests whose factorization completed, together: one
//      FGMRES over all their right-hand sides whose preconditioner applies
//      and SpMVs run one launch per phase for all of them (requests of very
//      different sizes in separate groups), and retires them.
#include <algorithm>
#include <deque>
#include <map>
#include <memory>

#include "engine.hpp"
#include "pool.hpp"

namespace spaqr {

struct Request {
  uint64_t ticket = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  spaqr_csr A{};
  Ordering ord;
  spaqr_opts opts{};
  std::vector<double> b, x;
  int64_t nrhs = 0;
  double tol = 1e-10;
  size_t est = 0;
  std::unique_ptr<Symbolic> sym;
  std::unique_ptr<EngineBase> eng;
  std::vector<spaqr_solve_info> info;
  int status = SPAQR_PENDING;
};

}  // namespace spaqr

struct spaqr_server {
  size_t budget = 0, used = 0;
  hipStream_t stream = nullptr;
  uint64_t next = 1;
  std::deque<std::unique_ptr<spaqr::Request>> queue;
  std::vector<std::unique_ptr<spaqr::Request>> active;
  std::map<uint64_t, std::unique_ptr<spaqr::Request>> done;
  spaqr::BatchDriver* drv = nullptr;
  std::unique_ptr<spaqr::HostPool> pool;  // admission of several requests in parallel
  ~spaqr_server() {
    active.clear();
    if (drv) spaqr::batch_driver_free(drv);
  }
};

using namespace spaqr;

namespace {
template <typename F>
spaqr_status guard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return e.status;
  } catch (const std::bad_alloc&) {
    return SPAQR_ENOMEM;
  } catch (...) {
    return SPAQR_EINVAL;
  }
}

void retire(spaqr_server* srv, std::unique_ptr<Request> r, int status) {
  r->status = status;
  r->eng.reset();
  r->sym.reset();
  srv->used -= r->est;
  srv->done[r->ticket] = std::move(r);
}

// Solves the factored requests rs together (one batched FGMRES: their
// preconditioner applies and SpMVs share launches), setting each one's
// status, x and info.
void solve_group(spaqr_server* srv, const std::vector<Request*>& rs, std::vector<int>& st) {
  const size_t np = rs.size();
  st.assign(np, SPAQR_OK);
  std::vector<EngineBase*> es;
  std::vector<int> nrhs;
  std::vector<const double*> db;
  std::vector<double*> dx;
  std::vector<double> tol;
  size_t tot = 0, cols = 0;
  for (Request* r : rs) tot += (size_t)r->A.n * r->nrhs;
  double* buf = static_cast<double*>(dev_alloc(std::max<size_t>(1, 2 * tot) * sizeof(double), srv->stream));
  try {
    size_t o = 0;
    for (Request* r : rs) {
      const size_t sz = (size_t)r->A.n * r->nrhs;
      SPAQR_HIP(hipMemcpyAsync(buf + o, r->b.data(), sz * sizeof(double), hipMemcpyHostToDevice, srv->stream));
      es.push_back(r->eng.get());
      nrhs.push_back((int)r->nrhs);
      db.push_back(buf + o);
      dx.push_back(buf + tot + o);
      tol.push_back(r->tol);
      cols += (size_t)r->nrhs;
      o += sz;
    }
    std::vector<spaqr_solve_info> info(cols);
    fgmres_solve_batch(es, nrhs, db, dx, tol, info.data(), &st);
    size_t c = 0;
    for (size_t i = 0; i < np; ++i) {
      Request& r = *rs[i];
      r.info.assign(info.begin() + c, info.begin() + c + r.nrhs);
      c += r.nrhs;
      r.x.resize((size_t)r.A.n * r.nrhs);
      SPAQR_HIP(hipMemcpyAsync(r.x.data(), dx[i], r.x.size() * sizeof(double), hipMemcpyDeviceToHost,
                               srv->stream));
    }
    SPAQR_HIP(hipStreamSynchronize(srv->stream));
  } catch (const Error& e) {
    (void)hipStreamSynchronize(srv->stream);
    st.assign(np, e.status);
  }
  dev_free(buf, srv->stream);
}

// Groups of factored requests solved together: sizes sorted descending, a
// group grows while the zero padding of its columns to the group's largest n
// stays below half of the padded vectors, its right-hand sides stay within
// kGroupCols and its padded vectors within kGroupElems entries (the Krylov
// bases of a group take about 2 (restart + 1) times that many doubles, and a
// group runs until its slowest column converges).
constexpr size_t kGroupCols = 64;
constexpr double kGroupElems = double(1 << 23);
std::vector<std::vector<Request*>> solve_groups(std::vector<Request*> rs) {
  std::sort(rs.begin(), rs.end(), [](const Request* a, const Request* b) { return a->A.n > b->A.n; });
  std::vector<std::vector<Request*>> g;
  double useful = 0, padded = 0;
  size_t cols = 0;
  for (Request* r : rs) {
    const double u = (double)r->A.n * r->nrhs;
    if (!g.empty()) {
      const double p = (double)g.back().front()->A.n * r->nrhs;
      if (2.0 * (useful + u) >= padded + p && cols + r->nrhs <= kGroupCols && padded + p <= kGroupElems) {
        g.back().push_back(r);
        useful += u;
        padded += p;
        cols += r->nrhs;
        continue;
      }
    }
    g.push_back({r});
    useful = padded = u;
    cols = r->nrhs;
  }
  return g;
}
}  // namespace

extern "C" {

spaqr_status spaqr_server_create(size_t mem_budget, void* hip_stream, spaqr_server** out) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(out && mem_budget > 0, SPAQR_EINVAL, "bad argument");
    auto* s = new spaqr_server();
    s->budget = mem_budget;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->drv = batch_driver_new();
    *out = s;
    return SPAQR_OK;
  });
}

spaqr_status spaqr_submit(spaqr_server* srv, const spaqr_csr* A, const spaqr_ordering* ord, const spaqr_opts* opts,
                          const double* b, int64_t nrhs, double tol, uint64_t* ticket) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(srv && A && ord && b && ticket && nrhs >= 1 && tol > 0, SPAQR_EINVAL, "bad argument");
    SPAQR_REQUIRE(A->n == ord->o.n, SPAQR_EINVAL, "matrix size differs from the ordering");
    auto r = std::make_unique<Request>();
    r->rowptr.assign(A->rowptr, A->rowptr + A->n + 1);
    r->col.assign(A->col, A->col + A->nnz);
    r->val.assign(A->val, A->val + A->nnz);
    r->A = {A->n, A->nnz, r->rowptr.data(), r->col.data(), r->val.data()};
    r->ord = ord->o;
    r->opts = opts ? *opts : spaqr_opts_default();
    r->b.assign(b, b + A->n * nrhs);
    r->nrhs = nrhs;
    r->tol = tol;
    SPAQR_REQUIRE(r->opts.precision == 32 || r->opts.precision == 64, SPAQR_EINVAL, "precision must be 32 or 64");
    // the symbolic analysis (host only) sizes the request: its admission
    // estimate is the analysis's bound on the device memory it can hold
    r->sym.reset(analyze(&r->A, r->ord, r->opts.skip));
    r->est = device_bytes_bound(*r->sym, r->opts.precision, nrhs, r->opts.restart);
    SPAQR_REQUIRE(r->est <= srv->budget, SPAQR_ENOMEM, "request alone exceeds the memory budget");
    r->ticket = srv->next++;
    *ticket = r->ticket;
    srv->queue.push_back(std::move(r));
    return SPAQR_OK;
  });
}

spaqr_status spaqr_server_step(spaqr_server* srv, int* active) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(srv, SPAQR_EINVAL, "NULL server");
    // 1. admission by estimated memory, in arrival order; the admitted
    // requests' set-ups run in parallel host threads
    std::vector<std::unique_ptr<Request>> adm;
    while (!srv->queue.empty() && srv->used + srv->queue.front()->est <= srv->budget) {
      adm.push_back(std::move(srv->queue.front()));
      srv->queue.pop_front();
      srv->used += adm.back()->est;
    }
    std::vector<int> adm_st(adm.size(), SPAQR_OK);
    if (!adm.empty()) {
      if (!srv->pool && adm.size() > 1) {
        srv->pool.reset(new HostPool(host_pool_threads()));
      }
      auto setup = [&](int i) {
        Request& r = *adm[i];
        try {
          r.eng = make_engine_deferred(&r.A, nullptr, *r.sym, r.opts, srv->stream);
        } catch (const Error& e) {
          adm_st[i] = e.status;
        } catch (const std::bad_alloc&) {
          adm_st[i] = SPAQR_ENOMEM;
        }
      };
      if (srv->pool) srv->pool->run((int)adm.size(), setup);
      else
        for (size_t i = 0; i < adm.size(); ++i) setup((int)i);
    }
    for (size_t i = 0; i < adm.size(); ++i) {
      if (adm_st[i] == SPAQR_OK) srv->active.push_back(std::move(adm[i]));
      else retire(srv, std::move(adm[i]), adm_st[i]);
    }
    // 2. one stage of every factoring request, batched across requests
    std::vector<EngineBase*> es;
    for (auto& r : srv->active)
      if (r->eng->stages_left() > 0) es.push_back(r->eng.get());
    if (!es.empty()) {
      try {
        factor_stage_batch(*srv->drv, es, srv->stream);
      } catch (const Error& e) {
        // a failure outside the per-request checks leaves the batch in an
        // unknown state: every request of it fails with that status
        (void)hipStreamSynchronize(srv->stream);
        std::vector<std::unique_ptr<Request>> keep;
        for (auto& r : srv->active) {
          if (r->eng->stages_left() > 0) retire(srv, std::move(r), e.status);
          else keep.push_back(std::move(r));
        }
        srv->active.swap(keep);
      }
    }
    // 3. solve the factored requests together and retire them
    std::vector<Request*> ready;
    for (auto& r : srv->active)
      if (r->eng->stages_left() == 0 && r->eng->error() == SPAQR_OK) ready.push_back(r.get());
    std::map<Request*, int> result;
    for (const auto& g : solve_groups(ready)) {
      std::vector<int> st;
      solve_group(srv, g, st);
      for (size_t i = 0; i < g.size(); ++i) result[g[i]] = st[i];
    }
    std::vector<std::unique_ptr<Request>> keep;
    for (auto& r : srv->active) {
      if (r->eng->stages_left() > 0) {
        keep.push_back(std::move(r));
        continue;
      }
      const int st = r->eng->error() != SPAQR_OK ? r->eng->error() : result[r.get()];
      retire(srv, std::move(r), st);
    }
    const bool retired = keep.size() < srv->active.size();
    srv->active.swap(keep);
    // requests of many sizes pass through one server: return what the
    // retired ones freed once the cache holds a large share of the device
    if (retired) mem_trim_if_large();
    if (active) *active = (int)(srv->active.size() + srv->queue.size());
    return SPAQR_OK;
  });
}

spaqr_status spaqr_poll(spaqr_server* srv, uint64_t ticket, double* x, spaqr_solve_info* info) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(srv, SPAQR_EINVAL, "NULL server");
    auto it = srv->done.find(ticket);
    if (it == srv->done.end()) return SPAQR_PENDING;
    Request& r = *it->second;
    if (x) std::copy(r.x.begin(), r.x.end(), x);
    if (info) std::copy(r.info.begin(), r.info.end(), info);
    const int st = r.status;
    srv->done.erase(it);
    return st;
  });
}

spaqr_status spaqr_server_status(const spaqr_server* srv, int64_t* queued, int64_t* resident, size_t* bytes) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(srv, SPAQR_EINVAL, "NULL server");
    if (queued) *queued = (int64_t)srv->queue.size();
    if (resident) *resident = (int64_t)srv->active.size();
    if (bytes) *bytes = srv->used;
    return SPAQR_OK;
  });
}

spaqr_status spaqr_estimate_bytes(const spaqr_symbolic* sym, const spaqr_opts* opts, int64_t nrhs, size_t* bytes) {
  return guard([&]() -> spaqr_status {
    SPAQR_REQUIRE(sym && bytes && nrhs >= 1, SPAQR_EINVAL, "bad argument");
    const spaqr_opts o = opts ? *opts : spaqr_opts_default();
    SPAQR_REQUIRE(o.precision == 32 || o.precision == 64, SPAQR_EINVAL, "precision must be 32 or 64");
    *bytes = device_bytes_bound(sym->s, o.precision, nrhs, o.restart);
    return SPAQR_OK;
  });
}

void spaqr_server_destroy(spaqr_server* srv) {
  try {
    delete srv;
  } catch (...) {
  }
}

}  // extern "C"
