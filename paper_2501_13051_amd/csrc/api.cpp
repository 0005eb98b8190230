// C ABI of libfv.so (declared in include/fv.h): argument checks and error
// translation around the host runtime.  No exception crosses this boundary.
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "engine.h"

struct fv_ctx {
  explicit fv_ctx(const fv_options* o) : eng(o) {}
  fv::Engine eng;
};

namespace {

template <typename F>
fv_status guarded(fv_ctx* ctx, F&& f) {
  if (!ctx) return FV_EINVAL;
  try {
    ctx->eng.last_error.clear();
    f();
    return FV_OK;
  } catch (const fv::Error& e) {
    ctx->eng.last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->eng.last_error = "host allocation failed";
    return FV_ENOMEM;
  } catch (const std::exception& e) {
    ctx->eng.last_error = e.what();
    return FV_EINVAL;
  }
}

}  // namespace

extern "C" {

fv_status fv_ctx_create(fv_ctx** out, const fv_options* opt) {
  if (!out) return FV_EINVAL;
  *out = nullptr;
  try {
    *out = new fv_ctx(opt);
    return FV_OK;
  } catch (const fv::Error& e) {
    return e.code;
  } catch (...) {
    return FV_ENOMEM;
  }
}

void fv_ctx_destroy(fv_ctx* ctx) { delete ctx; }

const char* fv_last_error(const fv_ctx* ctx) { return ctx ? ctx->eng.last_error.c_str() : "null context"; }

fv_status fv_relation_create(fv_ctx* ctx, const char* name, uint32_t arity, fv_rel* out) {
  if (!out) return FV_EINVAL;
  return guarded(ctx, [&] { *out = ctx->eng.relation_create(name, arity); });
}

fv_status fv_relation_find(fv_ctx* ctx, const char* name, fv_rel* out) {
  if (!out) return FV_EINVAL;
  return guarded(ctx, [&] { *out = ctx->eng.relation_find(name); });
}

fv_status fv_load_columns(fv_ctx* ctx, fv_rel rel, const uint32_t* const* cols, uint64_t n_rows, int on_device) {
  return guarded(ctx, [&] {
    if (ctx->eng.terminal) throw fv::Error(FV_ESTATE, "context is in an error state");
    ctx->eng.load_columns(rel, cols, n_rows, on_device != 0);
  });
}

fv_status fv_add_rule(fv_ctx* ctx, const fv_rule* rule) {
  return guarded(ctx, [&] {
    if (!rule) throw fv::Error(FV_EINVAL, "null rule");
    ctx->eng.add_rule(*rule);
  });
}

fv_status fv_run_fixpoint(fv_ctx* ctx, fv_stats* stats) {
  return guarded(ctx, [&] { ctx->eng.run(stats); });
}

fv_status fv_run_batch(fv_ctx* const* ctxs, uint32_t n, fv_stats* stats) {
  if (!ctxs || n == 0 || !ctxs[0]) return FV_EINVAL;
  std::vector<fv::Engine*> es(n);
  for (uint32_t k = 0; k < n; ++k) {
    if (!ctxs[k]) return FV_EINVAL;
    es[k] = &ctxs[k]->eng;
  }
  return guarded(ctxs[0], [&] { fv::Engine::run_batch(es.data(), n, stats); });
}

fv_status fv_relation_size(fv_ctx* ctx, fv_rel rel, uint64_t* n_rows) {
  if (!n_rows) return FV_EINVAL;
  return guarded(ctx, [&] { *n_rows = ctx->eng.relation_size(rel); });
}

fv_status fv_export(fv_ctx* ctx, fv_rel rel, uint32_t* const* cols_out, uint64_t capacity, uint64_t* n_rows_out,
                    int on_device) {
  return guarded(ctx, [&] {
    if (ctx->eng.terminal) throw fv::Error(FV_ESTATE, "context is in an error state");
    ctx->eng.export_rel(rel, cols_out, capacity, n_rows_out, on_device != 0);
  });
}

fv_status fv_delta_sizes(fv_ctx* ctx, uint64_t* out, uint32_t cap, uint32_t* n) {
  return guarded(ctx, [&] {
    const auto& d = ctx->eng.delta_sizes();
    if (n) *n = uint32_t(d.size());
    if (out)
      for (uint32_t i = 0; i < cap && i < d.size(); ++i) out[i] = d[i];
  });
}

fv_status fv_join_trace(fv_ctx* ctx, float* rows, uint32_t cap, uint32_t* n) {
  return guarded(ctx, [&] {
    const auto& t = ctx->eng.join_trace();
    const uint32_t cols = fv::Engine::kTraceCols;
    const uint32_t total = uint32_t(t.size() / cols);
    if (n) *n = total;
    if (rows)
      for (uint32_t i = 0; i < cap && i < total; ++i)
        for (uint32_t c = 0; c < cols; ++c) rows[size_t(i) * cols + c] = t[size_t(i) * cols + c];
  });
}

fv_status fv_profile(fv_ctx* ctx, fv_kprof* out, uint32_t cap, uint32_t* n) {
  return guarded(ctx, [&] {
    const auto& k = ctx->eng.profile();
    if (n) *n = uint32_t(k.size());
    if (out)
      for (uint32_t i = 0; i < cap && i < k.size(); ++i) {
        fv_kprof& o = out[i];
        std::snprintf(o.name, sizeof(o.name), "%s", k[i].name.c_str());
        o.launches = k[i].launches;
        o.ms = k[i].ms;
        o.algo_bytes = k[i].bytes;
        o.items = k[i].items;
      }
  });
}

}  // extern "C"
