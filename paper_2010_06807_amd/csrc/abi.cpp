// extern "C" entry points: argument checks, exception -> status translation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "engine.hpp"
#include "pool.hpp"
#include "profile.hpp"

using namespace spaqr;

namespace {

thread_local std::string g_last_error;

template <typename F>
spaqr_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SPAQR_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SPAQR_EINVAL;
  }
}

void require_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  SPAQR_REQUIRE(e == hipSuccess && n > 0, SPAQR_EDEVICE, "no HIP device available");
}

}  // namespace

extern "C" {

const char* spaqr_status_string(int s) {
  switch (s) {
    case SPAQR_OK: return "ok";
    case SPAQR_ENOCONV: return "GMRES did not converge within maxit";
    case SPAQR_PENDING: return "request pending";
    case SPAQR_EINVAL: return "invalid argument";
    case SPAQR_ENOMEM: return "out of memory";
    case SPAQR_ESINGULAR: return "exactly singular front";
    case SPAQR_EDEVICE: return "HIP device error";
    default: return "unknown status";
  }
}

const char* spaqr_last_error(void) { return g_last_error.c_str(); }

spaqr_status spaqr_order_grid(int dim, const int32_t sides[3], int nlevels, spaqr_ordering** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(sides && out, SPAQR_EINVAL, "NULL argument");
    std::unique_ptr<Ordering> o(build_grid_ordering(dim, sides, nlevels));
    auto* h = new spaqr_ordering();
    h->o = std::move(*o);
    *out = h;
    return SPAQR_OK;
  });
}

spaqr_status spaqr_order_graph(const spaqr_csr* A, int nlevels, spaqr_ordering** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(A && out && A->rowptr && A->col, SPAQR_EINVAL, "NULL argument");
    SPAQR_REQUIRE(A->n >= 1 && A->rowptr[0] == 0 && A->rowptr[A->n] == A->nnz, SPAQR_EINVAL,
                  "graph ordering: bad CSR row pointers");
    std::unique_ptr<Ordering> o(build_graph_ordering(A->n, A->rowptr, A->col, nlevels));
    auto* h = new spaqr_ordering();
    h->o = std::move(*o);
    *out = h;
    return SPAQR_OK;
  });
}

void spaqr_ordering_free(spaqr_ordering* o) { delete o; }

int64_t spaqr_ordering_n(const spaqr_ordering* o) { return o ? o->o.n : -1; }

int spaqr_ordering_levels(const spaqr_ordering* o) { return o ? o->o.L : -1; }

spaqr_status spaqr_ordering_perm(const spaqr_ordering* o, int64_t* perm) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(o && perm, SPAQR_EINVAL, "NULL argument");
    std::memcpy(perm, o->o.perm.data(), o->o.perm.size() * sizeof(int64_t));
    return SPAQR_OK;
  });
}

int64_t spaqr_ordering_num_clusters(const spaqr_ordering* o, int stage) {
  if (!o || stage < 1 || stage > o->o.L) return -1;
  return o->o.stages[stage].count();
}

spaqr_status spaqr_ordering_clusters(const spaqr_ordering* o, int stage, int64_t* start, int64_t* end,
                                     int64_t* node, int32_t* level) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(o && stage >= 1 && stage <= o->o.L, SPAQR_EINVAL, "bad stage");
    const StageClusters& c = o->o.stages[stage];
    const size_t n = (size_t)c.count();
    if (start) std::memcpy(start, c.start.data(), n * sizeof(int64_t));
    if (end) std::memcpy(end, c.end.data(), n * sizeof(int64_t));
    if (node) std::memcpy(node, c.node.data(), n * sizeof(int64_t));
    if (level) std::memcpy(level, c.level.data(), n * sizeof(int32_t));
    return SPAQR_OK;
  });
}

spaqr_status spaqr_ordering_merge_parents(const spaqr_ordering* o, int stage, int64_t* parent) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(o && parent && stage >= 2 && stage <= o->o.L, SPAQR_EINVAL, "bad stage");
    const StageClusters& c = o->o.stages[stage];
    std::memcpy(parent, c.parent.data(), c.parent.size() * sizeof(int64_t));
    return SPAQR_OK;
  });
}

spaqr_opts spaqr_opts_default(void) {
  spaqr_opts o;
  o.eps = 1e-2;
  o.skip = 2;
  o.scale = 1;
  o.precision = 32;
  o.restart = 100;
  o.maxit = 1000;
  return o;
}

spaqr_status spaqr_analyze(const spaqr_csr* A, const spaqr_ordering* ord, const spaqr_opts* opts,
                           spaqr_symbolic** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(A && ord && out, SPAQR_EINVAL, "NULL argument");
    const int skip = opts ? opts->skip : 2;
    std::unique_ptr<Symbolic> s(analyze(A, ord->o, skip));
    auto* h = new spaqr_symbolic();
    h->s = std::move(*s);
    *out = h;
    return SPAQR_OK;
  });
}

void spaqr_symbolic_free(spaqr_symbolic* s) { delete s; }

spaqr_status spaqr_symbolic_stage_info(const spaqr_symbolic* sym, int stage, int what, int32_t* buf,
                                       int64_t cap, int64_t* len) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(sym && len && stage >= 1 && stage <= sym->s.L, SPAQR_EINVAL, "bad argument");
    const StageSym& ss = sym->s.st[stage];
    std::vector<int32_t> v;
    if (what == 0 || what == 1) {
      for (const Pair& p : (what == 0 ? ss.in : ss.post).pairs()) {
        v.push_back(p.first);
        v.push_back(p.second);
      }
    } else if (what == 2) {
      for (const FrontSym& f : ss.fronts) {
        v.push_back(f.cluster);
        v.push_back(f.colour);
        v.push_back((int32_t)f.n1.size());
        v.insert(v.end(), f.n1.begin(), f.n1.end());
        v.push_back((int32_t)f.cols.size());
        v.insert(v.end(), f.cols.begin(), f.cols.end());
      }
    } else if (what == 3) {
      for (const IfaceSym& f : ss.ifaces) {
        v.push_back(f.cluster);
        v.push_back(f.colour);
      }
    } else {
      throw Error(SPAQR_EINVAL, "unknown info kind");
    }
    *len = (int64_t)v.size();
    if (buf) {
      SPAQR_REQUIRE(cap >= (int64_t)v.size(), SPAQR_EINVAL, "buffer too small");
      std::memcpy(buf, v.data(), v.size() * sizeof(int32_t));
    }
    return SPAQR_OK;
  });
}

static spaqr_status factor_impl(const spaqr_csr* A, const spaqr_csr_dev* Ad, const Symbolic& S,
                                const spaqr_opts* opts, void* stream, spaqr_handle** out,
                                std::unique_ptr<Symbolic> owned) {
  SPAQR_REQUIRE(out, SPAQR_EINVAL, "NULL output");
  require_device();
  spaqr_opts o = opts ? *opts : spaqr_opts_default();
  SPAQR_REQUIRE(o.restart >= 1 && o.maxit >= 1, SPAQR_EINVAL, "restart and maxit must be >= 1");
  SPAQR_REQUIRE(o.skip == S.skip, SPAQR_EINVAL, "skip differs from the symbolic analysis");
  auto h = std::unique_ptr<spaqr_handle>(new spaqr_handle());
  h->owned_sym = std::move(owned);
  const Symbolic& Sref = h->owned_sym ? *h->owned_sym : S;
  h->e = make_engine(A, Ad, Sref, o, reinterpret_cast<hipStream_t>(stream));
  *out = h.release();
  return SPAQR_OK;
}

spaqr_status spaqr_factor(const spaqr_csr* A, const spaqr_ordering* ord, const spaqr_opts* opts,
                          void* hip_stream, spaqr_handle** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(A && ord && out, SPAQR_EINVAL, "NULL argument");
    std::unique_ptr<Symbolic> s(analyze(A, ord->o, opts ? opts->skip : 2));
    const Symbolic& ref = *s;
    SPAQR_REQUIRE(A->val, SPAQR_EINVAL, "NULL values");
    return factor_impl(A, nullptr, ref, opts, hip_stream, out, std::move(s));
  });
}

spaqr_status spaqr_factor_symbolic(const spaqr_csr* A, const spaqr_symbolic* sym, const spaqr_opts* opts,
                                   void* hip_stream, spaqr_handle** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(A && sym && out, SPAQR_EINVAL, "NULL argument");
    SPAQR_REQUIRE(A->n == sym->s.n && A->nnz == sym->s.nnz, SPAQR_EINVAL, "matrix does not match the analysis");
    SPAQR_REQUIRE(A->val, SPAQR_EINVAL, "NULL values");
    return factor_impl(A, nullptr, sym->s, opts, hip_stream, out, nullptr);
  });
}

spaqr_status spaqr_factor_device(const spaqr_csr* A, const spaqr_csr_dev* Ad, const spaqr_symbolic* sym,
                                 const spaqr_opts* opts, void* hip_stream, spaqr_handle** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(A && Ad && sym && out && A->rowptr && A->col, SPAQR_EINVAL, "NULL argument");
    SPAQR_REQUIRE(Ad->rowptr && Ad->col && Ad->val, SPAQR_EINVAL, "NULL device array");
    SPAQR_REQUIRE(A->n == sym->s.n && A->nnz == sym->s.nnz, SPAQR_EINVAL, "matrix does not match the analysis");
    return factor_impl(A, Ad, sym->s, opts, hip_stream, out, nullptr);
  });
}

spaqr_status spaqr_factor_batch(int nprob, const spaqr_csr* const* A, const spaqr_csr_dev* const* Ad,
                                const spaqr_symbolic* const* sym, const spaqr_opts* opts, void* hip_stream,
                                spaqr_handle** out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(nprob >= 1 && A && sym && out, SPAQR_EINVAL, "NULL argument");
    for (int i = 0; i < nprob; ++i) out[i] = nullptr;
    require_device();
    const spaqr_opts o = opts ? *opts : spaqr_opts_default();
    SPAQR_REQUIRE(o.restart >= 1 && o.maxit >= 1, SPAQR_EINVAL, "restart and maxit must be >= 1");
    const hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    std::vector<std::unique_ptr<spaqr_handle>> hs(nprob);
    for (int i = 0; i < nprob; ++i) {
      const spaqr_csr* a = A[i];
      const spaqr_csr_dev* ad = Ad ? Ad[i] : nullptr;
      SPAQR_REQUIRE(a && sym[i] && a->rowptr && a->col, SPAQR_EINVAL, "NULL problem argument");
      SPAQR_REQUIRE(a->n == sym[i]->s.n && a->nnz == sym[i]->s.nnz, SPAQR_EINVAL,
                    "matrix does not match the analysis");
      SPAQR_REQUIRE(o.skip == sym[i]->s.skip, SPAQR_EINVAL, "skip differs from the symbolic analysis");
      if (ad) SPAQR_REQUIRE(ad->rowptr && ad->col && ad->val, SPAQR_EINVAL, "NULL device array");
      else SPAQR_REQUIRE(a->val, SPAQR_EINVAL, "NULL values");
      hs[i].reset(new spaqr_handle());
    }
    // set-up (uploads, column scaling, first pool) of the problems in parallel
    {
      HostScope hsetup("host_setup");
      HostPool pool(std::min(nprob - 1, host_pool_threads()));
      pool.run(nprob, [&](int i) {
        hs[i]->e = make_engine_deferred(A[i], Ad ? Ad[i] : nullptr, sym[i]->s, o, s);
      });
    }
    std::vector<EngineBase*> es;
    for (int i = 0; i < nprob; ++i) es.push_back(hs[i]->e.get());
    BatchDriver* drv = batch_driver_new();
    try {
      for (;;) {
        bool more = false;
        for (EngineBase* e : es) more = more || e->stages_left() > 0;
        if (!more) break;
        factor_stage_batch(*drv, es, s);
      }
    } catch (...) {
      batch_driver_free(drv);
      (void)hipStreamSynchronize(s);
      throw;
    }
    batch_driver_free(drv);
    {
      HostScope hsync("host_final_sync");
      SPAQR_HIP(hipStreamSynchronize(s));
    }
    spaqr_status st = SPAQR_OK;
    for (int i = 0; i < nprob; ++i) {
      const int err = hs[i]->e->error();
      if (err != SPAQR_OK) {
        if (st == SPAQR_OK) {
          st = err;
          g_last_error = std::string("problem ") + std::to_string(i) + ": " + hs[i]->e->error_message();
        }
        hs[i].reset();
      } else {
        out[i] = hs[i].release();
      }
    }
    return st;
  });
}

spaqr_status spaqr_solve_batch(int nprob, spaqr_handle* const* h, const double* const* b, double* const* x,
                               const int64_t* nrhs, int on_device, const double* tol, spaqr_solve_info* info) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(nprob >= 1 && h && b && x && nrhs && tol, SPAQR_EINVAL, "NULL argument");
    std::vector<EngineBase*> es;
    std::vector<int> nr;
    std::vector<double> tl;
    for (int i = 0; i < nprob; ++i) {
      SPAQR_REQUIRE(h[i] && b[i] && x[i], SPAQR_EINVAL, "NULL problem argument");
      SPAQR_REQUIRE(nrhs[i] >= 1 && nrhs[i] <= (1 << 16), SPAQR_EINVAL, "bad number of right-hand sides");
      SPAQR_REQUIRE(tol[i] > 0.0 && std::isfinite(tol[i]), SPAQR_EINVAL, "tol must be > 0");
      SPAQR_REQUIRE(!on_device || b[i] != x[i], SPAQR_EINVAL, "b and x must not alias");
      es.push_back(h[i]->e.get());
      nr.push_back((int)nrhs[i]);
      tl.push_back(tol[i]);
    }
    const hipStream_t s = es[0]->stream();
    if (on_device) {
      std::vector<const double*> db(b, b + nprob);
      std::vector<double*> dx(x, x + nprob);
      return fgmres_solve_batch(es, nr, db, dx, tl, info, nullptr);
    }
    size_t tot = 0;
    for (int i = 0; i < nprob; ++i) tot += (size_t)es[i]->n() * nr[i];
    double* buf = static_cast<double*>(dev_alloc(2 * tot * sizeof(double), s));
    std::vector<const double*> db;
    std::vector<double*> dx;
    size_t o = 0;
    for (int i = 0; i < nprob; ++i) {
      const size_t sz = (size_t)es[i]->n() * nr[i];
      db.push_back(buf + o);
      dx.push_back(buf + tot + o);
      o += sz;
    }
    int st;
    try {
      for (int i = 0; i < nprob; ++i)
        SPAQR_HIP(hipMemcpyAsync(const_cast<double*>(db[i]), b[i], (size_t)es[i]->n() * nr[i] * sizeof(double),
                                 hipMemcpyHostToDevice, s));
      st = fgmres_solve_batch(es, nr, db, dx, tl, info, nullptr);
      for (int i = 0; i < nprob; ++i)
        SPAQR_HIP(hipMemcpyAsync(x[i], dx[i], (size_t)es[i]->n() * nr[i] * sizeof(double), hipMemcpyDeviceToHost,
                                 s));
      SPAQR_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      dev_free(buf, s);
      throw;
    }
    dev_free(buf, s);
    return st;
  });
}

static void to_device(spaqr_handle* h, const double* b, int64_t nrhs, int64_t ld, double** db) {
  const int64_t N = h->e->n();
  *db = static_cast<double*>(dev_alloc((size_t)N * nrhs * sizeof(double), h->e->stream()));
  SPAQR_HIP(hipMemcpy2DAsync(*db, N * sizeof(double), b, ld * sizeof(double), N * sizeof(double), nrhs,
                             hipMemcpyHostToDevice, h->e->stream()));
}

spaqr_status spaqr_apply(spaqr_handle* h, const double* b, double* x, int64_t nrhs, int64_t ld, int on_device) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && b && x && nrhs >= 1 && ld >= h->e->n(), SPAQR_EINVAL, "bad argument");
    SPAQR_REQUIRE(nrhs <= (1 << 20), SPAQR_EINVAL, "too many right-hand sides");
    const int64_t N = h->e->n();
    hipStream_t s = h->e->stream();
    if (on_device) {
      h->e->apply_dev(b, ld, x, ld, (int)nrhs);
    } else {
      double* db = nullptr;
      to_device(h, b, nrhs, ld, &db);
      h->e->apply_dev(db, N, db, N, (int)nrhs);
      SPAQR_HIP(hipMemcpy2DAsync(x, ld * sizeof(double), db, N * sizeof(double), N * sizeof(double), nrhs,
                                 hipMemcpyDeviceToHost, s));
      dev_free(db, s);
    }
    SPAQR_HIP(hipStreamSynchronize(s));
    return SPAQR_OK;
  });
}

spaqr_status spaqr_solve(spaqr_handle* h, const double* b, double* x, int64_t nrhs, int64_t ld, int on_device,
                         double tol, spaqr_solve_info* info) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && b && x && nrhs >= 1 && ld >= h->e->n(), SPAQR_EINVAL, "bad argument");
    SPAQR_REQUIRE(tol > 0.0 && std::isfinite(tol), SPAQR_EINVAL, "tol must be > 0");
    const int64_t N = h->e->n();
    hipStream_t s = h->e->stream();
    int st;
    const std::vector<double> tv((size_t)nrhs, tol);
    EngineBase& e = *h->e;
    std::vector<double> hist;
    if (on_device) {
      SPAQR_REQUIRE(b != x, SPAQR_EINVAL, "b and x must not alias in spaqr_solve");
      st = fgmres_solve(e, b, ld, x, ld, (int)nrhs, tv.data(), e.opt_restart(), e.opt_maxit(), info, &hist);
    } else {
      double *db = nullptr, *dx = nullptr;
      to_device(h, b, nrhs, ld, &db);
      dx = static_cast<double*>(dev_alloc((size_t)N * nrhs * sizeof(double), s));
      st = fgmres_solve(e, db, N, dx, N, (int)nrhs, tv.data(), e.opt_restart(), e.opt_maxit(), info, &hist);
      SPAQR_HIP(hipMemcpy2DAsync(x, ld * sizeof(double), dx, N * sizeof(double), N * sizeof(double), nrhs,
                                 hipMemcpyDeviceToHost, s));
      dev_free(db, s);
      dev_free(dx, s);
    }
    SPAQR_HIP(hipStreamSynchronize(s));
    e.set_history(std::move(hist));
    return st;
  });
}

spaqr_status spaqr_stats(const spaqr_handle* h, spaqr_stats_t* out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && out, SPAQR_EINVAL, "NULL argument");
    *out = h->e->stats().s;
    return SPAQR_OK;
  });
}

spaqr_status spaqr_stage_sizes(const spaqr_handle* h, int stage, int32_t* buf, int64_t cap, int64_t* len) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && len, SPAQR_EINVAL, "NULL argument");
    const auto& ss = h->e->stats().stage_sizes;
    SPAQR_REQUIRE(stage >= 1 && stage < (int)ss.size(), SPAQR_EINVAL, "bad stage");
    *len = (int64_t)ss[stage].size();
    if (buf) {
      SPAQR_REQUIRE(cap >= *len, SPAQR_EINVAL, "buffer too small");
      std::memcpy(buf, ss[stage].data(), ss[stage].size() * sizeof(int32_t));
    }
    return SPAQR_OK;
  });
}

spaqr_status spaqr_stage_stats(const spaqr_handle* h, int stage, spaqr_stage_stats_t* out) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && out, SPAQR_EINVAL, "NULL argument");
    SPAQR_REQUIRE(h->e->stages_left() == 0 && h->e->error() == SPAQR_OK, SPAQR_EINVAL,
                  "the factorization is not complete");
    const auto& st = h->e->stats().stage;
    SPAQR_REQUIRE(stage >= 1 && stage < (int)st.size(), SPAQR_EINVAL, "bad stage");
    *out = st[stage];
    return SPAQR_OK;
  });
}

spaqr_status spaqr_stage_interfaces(const spaqr_handle* h, int stage, int32_t* buf, int64_t cap, int64_t* len) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && len, SPAQR_EINVAL, "NULL argument");
    const auto& fi = h->e->stats().ifaces;
    SPAQR_REQUIRE(stage >= 1 && stage < (int)fi.size(), SPAQR_EINVAL, "bad stage");
    *len = (int64_t)fi[stage].size();
    if (buf) {
      SPAQR_REQUIRE(cap >= *len, SPAQR_EINVAL, "buffer too small");
      std::memcpy(buf, fi[stage].data(), fi[stage].size() * sizeof(int32_t));
    }
    return SPAQR_OK;
  });
}

spaqr_status spaqr_solve_history(const spaqr_handle* h, double* buf, int64_t cap, int64_t* len) {
  return guarded([&]() -> spaqr_status {
    SPAQR_REQUIRE(h && len, SPAQR_EINVAL, "NULL argument");
    const auto& hi = h->e->stats().history;
    *len = (int64_t)hi.size();
    if (buf) {
      SPAQR_REQUIRE(cap >= *len, SPAQR_EINVAL, "buffer too small");
      std::memcpy(buf, hi.data(), hi.size() * sizeof(double));
    }
    return SPAQR_OK;
  });
}

void spaqr_prof_release();

void spaqr_finalize(void) {
  try {
    spaqr_prof_release();
    mem_release_all();
  } catch (...) {
  }
}

void spaqr_free(spaqr_handle* h) {
  try {
    delete h;
    spaqr::mem_trim_if_large();
  } catch (...) {
  }
}

}  // extern "C"
