// C-ABI entry points of libgeneo.  Every entry catches its exceptions and
// returns a geneo_status; the message goes to the context.
#include <cstring>

#include "model.h"

namespace geneo {
void build_topology(geneo_system* s, const geneo_mesh* m);
void assemble_device(geneo_ctx* ctx, geneo_system* s, const double* mu, const double* eps, double gamma);
void build_decomposition(const geneo_system* s, const geneo_partition_opts* o, geneo_decomp* dec);
void noalloc_init(int device);
void potrf_noalloc(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, const int64_t* off_host, void* A,
                   int32_t precision, double* elapsed_ms);
FactorConfig autotune_factor(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, int precision, int reps,
                             double* best_ms, int* tried);
}  // namespace geneo

using namespace geneo;

template <typename F>
static int guarded(geneo_ctx* ctx, F&& f) {
  try {
    if (ctx) HIP_CHECK(hipSetDevice(ctx->device));
    f();
    return GENEO_OK;
  } catch (const Error& e) {
    if (ctx) ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return GENEO_EOOM;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return GENEO_EINVAL;
  }
}

// message of the last failed geneo_create (no context to hold it)
static thread_local std::string g_create_err;

extern "C" {

int geneo_create(geneo_ctx** out, int device, void* hip_stream) {
  if (!out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_ctx* ctx = new (std::nothrow) geneo_ctx();
  if (!ctx) return GENEO_EOOM;
  ctx->device = device;
  int rc = guarded(ctx, [&] {
    int ndev = 0;
    HIP_CHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) throw Error(GENEO_EINVAL, "no such device");
    HIP_CHECK(hipSetDevice(device));
    noalloc_init(device);   // device address of the allocation-free entry's scratch array
    // NULL is the device's default (null) stream: work is then ordered with
    // everything else issued on it, e.g. torch's default stream.
    ctx->stream = (hipStream_t)hip_stream;
    HIP_CHECK(hipMalloc(&ctx->d_err, sizeof(DevErr)));
    HIP_CHECK(hipMemset(ctx->d_err, 0, sizeof(DevErr)));
    HIP_CHECK(hipHostMalloc((void**)&ctx->h_err, sizeof(DevErr), hipHostMallocDefault));
    HIP_CHECK(hipMalloc(&ctx->d_sync, 4 * sizeof(unsigned)));
    HIP_CHECK(hipMemset(ctx->d_sync, 0, 4 * sizeof(unsigned)));
    for (auto& e : ctx->ev) HIP_CHECK(hipEventCreate(&e));
  });
  if (rc != GENEO_OK) {
    g_create_err = ctx->err;
    geneo_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return GENEO_OK;
}

void geneo_destroy(geneo_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->d_err) (void)hipFree(ctx->d_err);
  if (ctx->h_err) (void)hipHostFree(ctx->h_err);
  if (ctx->d_sync) (void)hipFree(ctx->d_sync);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  // cached large blocks of this device go back to the device (blocks still
  // held by live handles of other contexts are not cached, so not touched)
  BlockPool::get().trim();
  delete ctx;
}

const char* geneo_last_error(const geneo_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int geneo_assemble(geneo_ctx* ctx, const geneo_mesh* mesh, const double* mu, const double* eps, double gamma,
                   geneo_system** out) {
  if (!ctx || !mesh || !mu || !eps || !out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_system* s = new (std::nothrow) geneo_system();
  if (!s) return GENEO_EOOM;
  int rc = guarded(ctx, [&] {
    if (mesh->n_nodes <= 0 || mesh->n_tets <= 0 || !mesh->xyz || !mesh->tets)
      throw Error(GENEO_EINVAL, "empty mesh");
    if (mesh->n_bfaces < 0 || (mesh->n_bfaces > 0 && !mesh->bfaces)) throw Error(GENEO_EINVAL, "bad boundary faces");
    build_topology(s, mesh);
    assemble_device(ctx, s, mu, eps, gamma);
  });
  if (rc != GENEO_OK) {
    delete s;
    return rc;
  }
  *out = s;
  return GENEO_OK;
}

int geneo_system_info_get(const geneo_system* s, geneo_system_info* info) {
  if (!s || !info) return GENEO_EINVAL;
  info->n = s->n;
  info->nnz = s->nnz;
  info->n_edges = s->n_edges;
  info->n_free_nodes = s->n_free_nodes;
  info->n_cells = s->n_cells;
  info->assemble_ms = s->assemble_ms;
  return GENEO_OK;
}

int geneo_system_export(geneo_ctx* ctx, const geneo_system* s, int32_t* rowptr, int32_t* colind, double* vals,
                        int32_t* free_edge_ids) {
  if (!ctx || !s) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    if (rowptr) std::memcpy(rowptr, s->rowptr.data(), sizeof(int32_t) * s->rowptr.size());
    if (colind) std::memcpy(colind, s->colind.data(), sizeof(int32_t) * s->colind.size());
    if (free_edge_ids) std::memcpy(free_edge_ids, s->free_edges.data(), sizeof(int32_t) * s->free_edges.size());
    if (vals) {
      HIP_CHECK(hipMemcpyAsync(vals, s->d_val.p, sizeof(double) * s->nnz, hipMemcpyDeviceToHost, ctx->stream));
      HIP_CHECK(hipStreamSynchronize(ctx->stream));
    }
  });
}

int geneo_spmv(geneo_ctx* ctx, const geneo_system* s, const double* x, double* y) {
  if (!ctx || !s || !x || !y) return GENEO_EINVAL;
  return guarded(ctx, [&] { launch_spmv(s, x, y, ctx->stream); HIP_CHECK(hipGetLastError()); });
}

int geneo_partition(geneo_ctx* ctx, const geneo_system* s, const geneo_partition_opts* o, geneo_decomp** out) {
  if (!ctx || !s || !o || !out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_decomp* d = new (std::nothrow) geneo_decomp();
  if (!d) return GENEO_EOOM;
  int rc = guarded(ctx, [&] { build_decomposition(s, o, d); });
  if (rc != GENEO_OK) {
    delete d;
    return rc;
  }
  *out = d;
  return GENEO_OK;
}

int geneo_decomp_info_get(const geneo_decomp* d, geneo_decomp_info* info) {
  if (!d || !info) return GENEO_EINVAL;
  info->n_sub = d->N;
  info->n_min = INT32_MAX;
  info->n_max = 0;
  info->sum_n = 0;
  info->sum_p = 0;
  info->n_floating = 0;
  info->sum_n3_over_3 = 0;
  for (int32_t i = 0; i < d->N; ++i) {
    int64_t ni = d->dofs_ptr[i + 1] - d->dofs_ptr[i];
    info->n_min = std::min<int32_t>(info->n_min, (int32_t)ni);
    info->n_max = std::max<int32_t>(info->n_max, (int32_t)ni);
    info->sum_n += ni;
    info->sum_p += d->p_all[i];
    info->n_floating += d->n_dropped[i] > 0;
    info->sum_n3_over_3 += (double)ni * ni * ni / 3.0;
  }
  return GENEO_OK;
}

int geneo_decomp_subdomain(const geneo_decomp* d, int32_t i, int32_t* n_i, int32_t* dofs, double* pou, int32_t* p_i,
                           int32_t* gnodes) {
  if (!d || i < 0 || i >= d->N) return GENEO_EINVAL;
  const int64_t b = d->dofs_ptr[i], e = d->dofs_ptr[i + 1];
  if (n_i) *n_i = (int32_t)(e - b);
  if (dofs) std::memcpy(dofs, d->dofs.data() + b, sizeof(int32_t) * (e - b));
  if (pou) std::memcpy(pou, d->pou.data() + b, sizeof(double) * (e - b));
  const int64_t gb = d->gn_ptr[i], ge = d->gn_ptr[i + 1];
  if (p_i) *p_i = (int32_t)(ge - gb);
  if (gnodes) std::memcpy(gnodes, d->gnodes.data() + gb, sizeof(int32_t) * (ge - gb));
  return GENEO_OK;
}

void geneo_setup_opts_default(geneo_setup_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau = 10.0;
  o->nev_max = 20;
  o->coarse = GENEO_COARSE_SNK_GENEO;
  o->local_precision = GENEO_FP64;
  o->lobpcg_tol = 1e-8;
  o->lobpcg_maxit = 100;
  o->lobpcg_guard = 4;
  o->seed = 12345;
  o->coarse_drop_tol = 1e-7;
  o->warm_start = nullptr;
  o->fp32_rho_max = 0.5;
  o->model = nullptr;
  o->keep_ritz = 0;
  o->coarse_order = GENEO_ORDER_AUTO;
}

int geneo_setup(geneo_ctx* ctx, const geneo_system* s, const geneo_decomp* d, const geneo_setup_opts* o,
                geneo_precond** out) {
  if (!ctx || !s || !d || !out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_precond* pc = new (std::nothrow) geneo_precond();
  if (!pc) return GENEO_EOOM;
  int rc = guarded(ctx, [&] {
    pc->sys = s;
    pc->dec = d;
    if (o)
      pc->opts = *o;
    else
      geneo_setup_opts_default(&pc->opts);
    if (!(pc->opts.tau > 0) || pc->opts.nev_max < 0 || !(pc->opts.coarse_drop_tol >= 0) ||
        !(pc->opts.fp32_rho_max >= 0 && pc->opts.fp32_rho_max < 1))
      throw Error(GENEO_EINVAL, "bad setup options");
    setup_precond(ctx, pc);
  });
  if (rc != GENEO_OK) {
    delete pc;
    return rc;
  }
  *out = pc;
  return GENEO_OK;
}

int geneo_precond_info_get(const geneo_precond* pc, geneo_precond_info* info) {
  if (!pc || !info) return GENEO_EINVAL;
  *info = pc->info;
  return GENEO_OK;
}

int geneo_precond_eigs(const geneo_precond* pc, int32_t i, double* lam, int32_t cap, int32_t* count,
                       int32_t* selected) {
  if (!pc || i < 0 || i >= pc->N) return GENEO_EINVAL;
  const auto& e = pc->eigs[i];
  int32_t c = (int32_t)std::min<size_t>(e.size(), (size_t)std::max(cap, 0));
  if (lam) std::memcpy(lam, e.data(), sizeof(double) * c);
  if (count) *count = c;
  if (selected) *selected = pc->eig_sel[i];
  return GENEO_OK;
}

int geneo_precond_ritz(geneo_ctx* ctx, const geneo_precond* pc, int32_t i, double* V, int32_t cap,
                       int32_t* k_out) {
  if (!ctx || !pc || i < 0 || i >= pc->N || cap < 0) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    if (!pc->d_ritz.p) throw Error(GENEO_EINVAL, "setup without keep_ritz = 1");
    const int32_t k = std::min(cap, pc->ritz_k);
    const int64_t ni = pc->dec->dofs_ptr[i + 1] - pc->dec->dofs_ptr[i];
    const int64_t ld = pc->voff[i + 1] - pc->voff[i];
    if (V)
      for (int32_t q = 0; q < k; ++q)
        HIP_CHECK(hipMemcpyAsync(V + (int64_t)q * ni, pc->d_ritz.p + pc->voff[i] * pc->ritz_k + (int64_t)q * ld,
                                 sizeof(double) * ni, hipMemcpyDeviceToHost, ctx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->stream));
    if (k_out) *k_out = k;
  });
}

int geneo_apply(geneo_ctx* ctx, const geneo_precond* pc, const double* r, double* z) {
  if (!ctx || !pc || !r || !z) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    apply_precond(ctx, pc, r, z);
    HIP_CHECK(hipGetLastError());
    check_device_error(ctx);
  });
}

int geneo_solve(geneo_ctx* ctx, const geneo_system* s, const geneo_precond* pc, const double* b, double* x,
                const geneo_solve_opts* o, geneo_solve_info* info) {
  if (!ctx || !s || !b || !x || !info) return GENEO_EINVAL;
  geneo_solve_opts def{1e-8, 1000, 1, GENEO_SOLVER_PCG, 0, 0, GENEO_PCG_DEFLATED};
  const geneo_solve_opts* op = o ? o : &def;
  if (!(op->rtol > 0) || op->maxit < 1 || op->restart < 0) return GENEO_EINVAL;
  if (op->pcg_form != GENEO_PCG_DEFLATED && op->pcg_form != GENEO_PCG_BALANCED) return GENEO_EINVAL;
  if (op->method != GENEO_SOLVER_PCG && op->method != GENEO_SOLVER_GMRES) return GENEO_EINVAL;
  std::memset(info, 0, sizeof(*info));
  return guarded(ctx, [&] {
    if (pc && pc->sys != s) throw Error(GENEO_EINVAL, "the preconditioner was built on another system");
    if (op->method == GENEO_SOLVER_GMRES)
      gmres(ctx, s, pc, b, x, op, info);
    else
      pcg(ctx, s, pc, b, x, op, info);
  });
}

int geneo_potrf_batched(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, const int64_t* off_host, void* A,
                        int32_t precision, double* elapsed_ms) {
  if (!ctx || batch < 1 || !n_host || !off_host || !A) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    std::vector<MatDesc> descs(batch);
    int64_t inv_off = 0;
    int32_t flag_off = 0;
    for (int32_t i = 0; i < batch; ++i) {
      if (n_host[i] < 1 || off_host[i] < 0 || off_host[i] % 32) throw Error(GENEO_EINVAL, "bad matrix size/offset");
      int64_t np = round_up(n_host[i], NB);
      descs[i] = MatDesc{off_host[i], inv_off, -1, 0, (int32_t)np, (int32_t)(np / NB), flag_off, n_host[i]};
      inv_off += 2 * np * NB;
      flag_off += (int32_t)(np / NB);
    }
    FactorPlan P;
    P.build(descs, ctx->stream, precision);
    HIP_CHECK(hipEventRecord(ctx->ev[0], ctx->stream));
    if (precision == GENEO_FP64) {
      DevBuf<double> inv;
      inv.alloc(inv_off);
      HIP_CHECK(hipEventRecord(ctx->ev[0], ctx->stream));
      factor(P, (double*)A, inv.p, nullptr, 0.0, nullptr, ctx->d_err, ctx->stream, nullptr, false);
      HIP_CHECK(hipEventRecord(ctx->ev[1], ctx->stream));
      HIP_CHECK(hipEventSynchronize(ctx->ev[1]));
    } else if (precision == GENEO_FP32_REFINE1) {
      DevBuf<float> inv;
      inv.alloc(inv_off);
      HIP_CHECK(hipEventRecord(ctx->ev[0], ctx->stream));
      factor(P, (float*)A, inv.p, nullptr, 0.0, nullptr, ctx->d_err, ctx->stream, nullptr, false);
      HIP_CHECK(hipEventRecord(ctx->ev[1], ctx->stream));
      HIP_CHECK(hipEventSynchronize(ctx->ev[1]));
    } else {
      throw Error(GENEO_EINVAL, "unknown precision");
    }
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
    if (elapsed_ms) *elapsed_ms = ms;
    check_device_error(ctx);
  });
}

int geneo_tune_factor(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, int32_t precision, int32_t reps,
                      geneo_factor_schedule* best, int32_t* tried) {
  if (!ctx || batch < 1 || !n_host || !best || reps < 1) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    double ms = 0;
    int nt = 0;
    const FactorConfig c = autotune_factor(ctx, batch, n_host, precision, reps, &ms, &nt);
    *best = geneo_factor_schedule{c.mode, c.group, c.rec_potrf, ms};
    if (tried) *tried = nt;
  });
}

int geneo_tune_lookup(int32_t batch, const int32_t* n_host, int32_t precision, geneo_factor_schedule* out) {
  if (batch < 1 || !n_host || !out) return GENEO_EINVAL;
  if (precision != GENEO_FP64 && precision != GENEO_FP32_REFINE1) return GENEO_EINVAL;
  int32_t max_blk = 0;
  for (int32_t i = 0; i < batch; ++i) {
    if (n_host[i] < 1) return GENEO_EINVAL;
    max_blk = std::max<int32_t>(max_blk, (int32_t)(round_up(n_host[i], NB) / NB));
  }
  const FactorConfig c = tuned_factor_config(precision, max_blk, batch);
  *out = geneo_factor_schedule{c.mode, c.group, c.rec_potrf, 0.0};
  return GENEO_OK;
}

int geneo_tune_save(const char* path) {
  if (!path) return GENEO_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return GENEO_EINVAL;
  const std::string t = tune_db_text();
  const bool ok = std::fwrite(t.data(), 1, t.size(), f) == t.size();
  return std::fclose(f) == 0 && ok ? GENEO_OK : GENEO_EINVAL;
}

int geneo_tune_load(const char* path) {
  if (!path) return GENEO_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return GENEO_EINVAL;
  std::string t;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) t.append(buf, k);
  std::fclose(f);
  try {
    tune_db_parse(t);
  } catch (const std::exception&) {
    return GENEO_EINVAL;
  }
  return GENEO_OK;
}

int geneo_potrf_batched_noalloc(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, const int64_t* off_host,
                                void* A, int32_t precision, double* elapsed_ms) {
  if (!ctx || batch < 1 || !n_host || !off_host || !A) return GENEO_EINVAL;
  return guarded(ctx, [&] {
    potrf_noalloc(ctx, batch, n_host, off_host, A, precision, elapsed_ms);
    check_device_error(ctx);
  });
}

void geneo_model_opts_default(geneo_model_opts* o) {
  if (!o) return;
  o->canvas = 12;
  o->hidden = 256;
  o->k = 20;
  o->seed = 2311;
}

int geneo_model_create(geneo_ctx* ctx, const geneo_model_opts* o, geneo_model** out) {
  if (!ctx || !out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_model_opts d;
  geneo_model_opts_default(&d);
  geneo_model* m = new (std::nothrow) geneo_model();
  if (!m) return GENEO_EOOM;
  int rc = guarded(ctx, [&] { model_init(m, o ? o : &d, ctx->stream); });
  if (rc != GENEO_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return GENEO_OK;
}

int geneo_model_info_get(const geneo_model* m, geneo_model_info* info) {
  if (!m || !info) return GENEO_EINVAL;
  info->in_dim = m->in_dim;
  info->rows = m->rows;
  info->k = m->k;
  info->hidden = m->hidden;
  info->canvas = m->C;
  info->n_params = model_n_params(m);
  int32_t h = 0;
  for (uint8_t x : m->holdout) h += x;
  info->n_holdout = h;
  info->n_train = (int32_t)m->holdout.size() - h;
  return GENEO_OK;
}

int geneo_model_collect(geneo_ctx* ctx, geneo_model* m, const geneo_system* s, const geneo_decomp* d,
                        const geneo_precond* pc, int32_t holdout) {
  if (!ctx || !m || !s || !d || !pc) return GENEO_EINVAL;
  return guarded(ctx, [&] { model_collect(ctx, m, s, d, pc, holdout); });
}

int geneo_model_train(geneo_ctx* ctx, geneo_model* m, const geneo_train_opts* o, geneo_train_info* info) {
  if (!ctx || !m || !o || !info) return GENEO_EINVAL;
  return guarded(ctx, [&] { model_train(ctx, m, o, info); });
}

int geneo_model_predict(geneo_ctx* ctx, const geneo_model* m, int32_t batch, const float* X, float* Y) {
  if (!ctx || !m || !X || !Y) return GENEO_EINVAL;
  return guarded(ctx, [&] { model_predict(ctx, m, batch, X, Y); });
}

int geneo_model_loss_grad(geneo_ctx* ctx, const geneo_model* m, int32_t batch, const float* X, const float* V,
                          const uint8_t* mask, double* loss, float* grad) {
  if (!ctx || !m || !X || !V || !mask || !loss) return GENEO_EINVAL;
  return guarded(ctx, [&] { *loss = model_loss_grad(ctx, m, batch, X, V, mask, grad); });
}

int geneo_model_get_params(const geneo_model* m, float* params) {
  if (!m || !params) return GENEO_EINVAL;
  return guarded(nullptr, [&] { model_get_params(m, params); });
}

int geneo_model_set_params(geneo_ctx* ctx, geneo_model* m, const float* params) {
  if (!ctx || !m || !params) return GENEO_EINVAL;
  return guarded(ctx, [&] { model_set_params(ctx, m, params, true); });
}

int geneo_model_save(const geneo_model* m, const char* path) {
  if (!m || !path) return GENEO_EINVAL;
  return guarded(nullptr, [&] { model_save(m, path); });
}

int geneo_model_load(geneo_ctx* ctx, const char* path, geneo_model** out) {
  if (!ctx || !path || !out) return GENEO_EINVAL;
  *out = nullptr;
  geneo_model* m = new (std::nothrow) geneo_model();
  if (!m) return GENEO_EOOM;
  int rc = guarded(ctx, [&] { model_load(ctx, m, path); });
  if (rc != GENEO_OK) {
    delete m;
    return rc;
  }
  *out = m;
  return GENEO_OK;
}

void geneo_free_model(geneo_model* m) { delete m; }

void geneo_free_system(geneo_system* s) { delete s; }
void geneo_free_decomp(geneo_decomp* d) { delete d; }
void geneo_free_precond(geneo_precond* pc) { delete pc; }

}  // extern "C"
