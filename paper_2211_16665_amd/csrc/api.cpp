// C ABI of the library: argument checks, error translation (no exception
// crosses the boundary) and the thread-local last-error message.
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "fwdem_internal.hpp"

using namespace fwdem;

static thread_local std::string g_err;

template <typename F>
static fwd_status guard(F &&f) {
  try {
    g_err.clear();
    f();
    return FWD_OK;
  } catch (const Error &e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return FWD_ERR_OOM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return FWD_ERR_INVALID_ARG;
  } catch (...) {
    g_err = "unknown error";
    return FWD_ERR_INVALID_ARG;
  }
}

static Plan &P(fwd_plan *h) {
  if (!h || !h->p) fail(FWD_ERR_INVALID_ARG, "plan is NULL");
  return *h->p;
}
static const Plan &P(const fwd_plan *h) {
  if (!h || !h->p) fail(FWD_ERR_INVALID_ARG, "plan is NULL");
  return *h->p;
}

// Device buffers the library carves (workspace, volume transform, scratch,
// snapshots) start on a 256-byte boundary, as hipMalloc returns them.
static void need_aligned(const void *ptr, const char *what) {
  if (reinterpret_cast<uintptr_t>(ptr) & 255u)
    fail(FWD_ERR_INVALID_ARG, std::string(what) + " must be 256-byte aligned");
}

// A buffer shorter than what the call reads or writes is refused before
// any device work.
static void need_bytes(size_t have, size_t need, const char *what) {
  if (have < need)
    fail(FWD_ERR_INVALID_ARG, std::string(what) + " of " + std::to_string(have) +
                                  " bytes, the call needs " + std::to_string(need));
}

extern "C" {

const char *fwd_last_error(void) { return g_err.c_str(); }

fwd_status fwd_plan_create(const fwd_plan_desc *desc, fwd_plan **out) {
  return guard([&] {
    if (!out) fail(FWD_ERR_INVALID_ARG, "plan_out is NULL");
    *out = nullptr;
    Plan *p = plan_create(desc);
    *out = new fwd_plan{p};
  });
}

void fwd_plan_destroy(fwd_plan *h) {
  if (!h) return;
  if (h->p) {
    try {
      dev_release(*h->p);
    } catch (...) {
    }
    delete h->p;
  }
  delete h;
}

fwd_status fwd_set_model(fwd_plan *h, const double *rho) {
  return guard([&] { set_model(P(h), rho); });
}

fwd_status fwd_set_model_vti(fwd_plan *h, const double *rho_h, const double *rho_v) {
  return guard([&] {
    if (!rho_v) fail(FWD_ERR_INVALID_ARG, "rho_v is NULL");
    set_model(P(h), rho_h, rho_v);
  });
}

fwd_status fwd_get_info(const fwd_plan *h, fwd_info *info) {
  return guard([&] {
    const Plan &p = P(h);
    if (!info) fail(FWD_ERR_INVALID_ARG, "info is NULL");
    std::memset(info, 0, sizeof *info);
    info->nx = p.nx;
    info->ny = p.ny;
    info->nz = p.nz;
    info->px = p.PX;
    info->have_basis = p.have_basis;
    info->basis_iters = p.basis_iters;
    info->basis_gamma = p.gamma;
    info->basis_fit = p.fit;
    if (!p.have_model) return;
    info->dt = p.dt;
    info->dt_cfl = p.dt_cfl;
    info->nt = p.nt;
    info->vmax = p.vmax;
    info->vref = p.vref;
    info->tau = p.tau;
    info->t0 = p.t0;
    info->src_scale = p.src_scale;
    info->n_rec_nodes = (int)p.rn_c.size();
    info->n_src_entries = (int)p.src_tg.size();
    info->n_adj_targets = (int)p.rn_c.size() * p.ns;
    info->workspace_bytes_forward = p.workspace_bytes(FWD_MODE_FORWARD);
    info->workspace_bytes_adjoint = p.workspace_bytes(FWD_MODE_ADJOINT);
    info->volume_bytes = p.volume_bytes();
    info->state_bytes = p.state_bytes();
  });
}

fwd_status fwd_get_table(const fwd_plan *h, int which, double *out, size_t n) {
  return guard([&] {
    if (!out) fail(FWD_ERR_INVALID_ARG, "out is NULL");
    get_table(P(h), which, out, n);
  });
}

fwd_status fwd_workspace_size(const fwd_plan *h, int mode, size_t *bytes) {
  return guard([&] {
    const Plan &p = P(h);
    if (!bytes) fail(FWD_ERR_INVALID_ARG, "bytes is NULL");
    if (mode != FWD_MODE_FORWARD && mode != FWD_MODE_ADJOINT) fail(FWD_ERR_INVALID_ARG, "mode");
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    *bytes = p.workspace_bytes(mode);
  });
}

fwd_status fwd_volume_size(const fwd_plan *h, size_t *bytes) {
  return guard([&] {
    const Plan &p = P(h);
    if (!bytes) fail(FWD_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = p.volume_bytes();
  });
}

fwd_status fwd_forward(fwd_plan *h, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                       double *E_rec, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !E_rec) fail(FWD_ERR_INVALID_ARG, "workspace and E_rec are required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    dev_forward(p, ws, ws_bytes, vol, vol_bytes, E_rec, stream);
  });
}

fwd_status fwd_forward_static(fwd_plan *h, void *vol, size_t vol_bytes, double *E_rec,
                              void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!E_rec) fail(FWD_ERR_INVALID_ARG, "E_rec is required");
    need_aligned(vol, "volume buffer");
    dev_forward_static(p, vol, vol_bytes, E_rec, stream);
  });
}

fwd_status fwd_run_begin(fwd_plan *h, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                         void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws) fail(FWD_ERR_INVALID_ARG, "workspace is required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    dev_run_begin(p, ws, ws_bytes, vol, vol_bytes, stream);
  });
}

fwd_status fwd_run_steps(fwd_plan *h, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                         int nsteps, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws) fail(FWD_ERR_INVALID_ARG, "workspace is required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    need_bytes(ws_bytes, p.workspace_bytes(FWD_MODE_FORWARD), "workspace");
    if (vol) need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    dev_run_steps(p, ws, vol, nsteps, stream);
  });
}

fwd_status fwd_run_receivers(fwd_plan *h, void *ws, size_t ws_bytes, double *E_rec,
                             void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !E_rec) fail(FWD_ERR_INVALID_ARG, "workspace and E_rec are required");
    need_aligned(ws, "workspace");
    need_bytes(ws_bytes, p.workspace_bytes(FWD_MODE_FORWARD), "workspace");
    dev_run_receivers(p, ws, E_rec, stream);
  });
}

fwd_status fwd_run_flush(fwd_plan *h, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                         void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws) fail(FWD_ERR_INVALID_ARG, "workspace is required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    need_bytes(ws_bytes, p.workspace_bytes(FWD_MODE_FORWARD), "workspace");
    if (vol) need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    if (vol) dev_run_flush(p, ws, vol, stream);
  });
}

fwd_status fwd_checkpoint_size(const fwd_plan *h, int with_volume, size_t *bytes) {
  return guard([&] {
    const Plan &p = P(h);
    if (!bytes) fail(FWD_ERR_INVALID_ARG, "bytes is NULL");
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    *bytes = p.state_bytes() + (with_volume ? p.volume_bytes() : 0);
  });
}

fwd_status fwd_checkpoint_save(fwd_plan *h, const void *ws, size_t ws_bytes, const void *vol,
                               size_t vol_bytes, void *snap, size_t snap_bytes, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !snap) fail(FWD_ERR_INVALID_ARG, "workspace and snapshot are required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    need_aligned(snap, "snapshot");
    need_bytes(ws_bytes, p.state_bytes(), "workspace");
    if (vol) need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    need_bytes(snap_bytes, p.state_bytes() + (vol ? p.volume_bytes() : 0), "snapshot");
    dev_checkpoint(p, ws, vol, snap, 1, stream);
  });
}

fwd_status fwd_checkpoint_restore(fwd_plan *h, void *ws, size_t ws_bytes, void *vol,
                                  size_t vol_bytes, const void *snap, size_t snap_bytes,
                                  void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !snap) fail(FWD_ERR_INVALID_ARG, "workspace and snapshot are required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    need_aligned(snap, "snapshot");
    need_bytes(ws_bytes, p.state_bytes(), "workspace");
    if (vol) need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    need_bytes(snap_bytes, p.state_bytes() + (vol ? p.volume_bytes() : 0), "snapshot");
    dev_checkpoint(p, ws, vol, const_cast<void *>(snap), 0, stream);
  });
}

fwd_status fwd_volume_export(fwd_plan *h, const void *vol, size_t vol_bytes, double *out,
                             void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!vol || !out) fail(FWD_ERR_INVALID_ARG, "volume and output are required");
    need_aligned(vol, "volume buffer");
    need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    dev_volume_export(p, vol, out, stream);
  });
}

fwd_status fwd_basis_build(fwd_plan *h, double gamma_rel, double gamma_abs, int max_iter,
                           double tol, double *fit_err, int *iters) {
  return guard([&] { basis_build(P(h), gamma_rel, gamma_abs, max_iter, tol, fit_err, iters); });
}

fwd_status fwd_adjoint(fwd_plan *h, void *ws, size_t ws_bytes, const void *vol,
                       size_t vol_bytes, const double *resid, double *grad, int accumulate,
                       double *E_adj, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !resid || !grad) fail(FWD_ERR_INVALID_ARG, "workspace, residual and gradient are required");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    if (vol) need_bytes(vol_bytes, p.volume_bytes(), "volume buffer");
    dev_adjoint(p, ws, ws_bytes, vol, resid, grad, accumulate, E_adj, stream);
  });
}

fwd_status fwd_adjoint_td_size(const fwd_plan *h, int segment, size_t *bytes) {
  return guard([&] {
    const Plan &p = P(h);
    if (!bytes) fail(FWD_ERR_INVALID_ARG, "bytes is NULL");
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (segment < 1) fail(FWD_ERR_INVALID_ARG, "segment must be >= 1");
    *bytes = p.td_scratch_bytes(segment);
  });
}

fwd_status fwd_adjoint_td(fwd_plan *h, void *ws, size_t ws_bytes, void *scratch,
                          size_t scratch_bytes, int segment, const double *resid, double *grad,
                          int accumulate, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws || !scratch || !resid || !grad)
      fail(FWD_ERR_INVALID_ARG, "workspace, scratch, residual and gradient are required");
    need_aligned(ws, "workspace");
    need_aligned(scratch, "scratch");
    dev_adjoint_td(p, ws, ws_bytes, scratch, scratch_bytes, segment, resid, grad, accumulate,
                   stream);
  });
}

fwd_status fwd_set_option(fwd_plan *h, int key, double value) {
  return guard([&] {
    Plan &p = P(h);
    const int v = (int)value;
    switch (key) {
      case FWD_OPT_GRAPH_STEPS:
        if (v < 0 || v > 4096) fail(FWD_ERR_INVALID_ARG, "graph steps in [0, 4096]");
        p.graph_steps = v;
        break;
      case FWD_OPT_BLOCK_X:
        if (v != 16 && v != 32 && v != 64 && v != 128 && v != 256)
          fail(FWD_ERR_INVALID_ARG, "block x in {16,32,64,128,256}");
        p.bx = v;
        break;
      case FWD_OPT_BLOCK_Y:
        if (v != 1 && v != 2 && v != 4 && v != 8 && v != 16)
          fail(FWD_ERR_INVALID_ARG, "block y in {1,2,4,8,16}");
        p.by = v;
        break;
      case FWD_OPT_XCD_REMAP:
        p.xcd = v ? 1 : 0;
        break;
      case FWD_OPT_SAMPLE_EVERY:
        if (v < 0) fail(FWD_ERR_INVALID_ARG, "sample interval >= 0");
        dev_set_sampling(p, v);
        break;
      case FWD_OPT_STRICT_CFL:
        p.strict_cfl = v ? 1 : 0;
        break;
      case FWD_OPT_DFT_BLOCK:
        if (v != 1 && v != 2 && v != 4 && v != 8 && v != 16 && v != 32)
          fail(FWD_ERR_INVALID_ARG, "transform block in {1,2,4,8,16,32}");
        p.kb = v;
        break;

      case FWD_OPT_VECTOR:
        if (v != 1 && v != 4) fail(FWD_ERR_INVALID_ARG, "vector option in {1, 4}");
        if (v != 1 && p.fd_order == 4) fail(FWD_ERR_INVALID_ARG, "order 4 runs with vector 1");
        p.vx = v;
        break;
      case FWD_OPT_SCHEDULE:
        if (v != 0 && v != 1 && v != 2) fail(FWD_ERR_INVALID_ARG, "schedule option in {0, 1, 2}");
        if (v != 0 && p.fd_order == 4) fail(FWD_ERR_INVALID_ARG, "order 4 runs with schedule 0");
        p.sched = v;
        break;
      case FWD_OPT_BARRIER_US:
        if (!(value >= 0.0)) fail(FWD_ERR_INVALID_ARG, "barrier wait limit >= 0 microseconds");
        p.barrier_us = value;
        break;
      case FWD_OPT_DFT_DECIMATE: {
        int l = 0;
        while (l <= 6 && (1 << l) != v) ++l;
        if (l > 6) fail(FWD_ERR_INVALID_ARG, "decimation in {1, 2, 4, ..., 64}");
        p.dec = v;
        p.dec_log2 = l;
        break;
      }
      case FWD_OPT_PERSIST_BLOCKS:
        if (v < 0 || v > 32) fail(FWD_ERR_INVALID_ARG, "blocks per compute unit in [0, 32]");
        p.persist_blocks = v;
        break;
      case FWD_OPT_BARRIER_SLEEP:
        if (v < 1 || v > 64) fail(FWD_ERR_INVALID_ARG, "barrier pause in [1, 64]");
        p.barrier_sleep = v;
        break;
      case FWD_OPT_STREAM_STORES:
        if (v < -1 || v > 1) fail(FWD_ERR_INVALID_ARG, "stream stores in {-1, 0, 1}");
        p.stream_stores = v;
        break;
      case FWD_OPT_ZCHUNK:
        if (v < 1 || v > 64) fail(FWD_ERR_INVALID_ARG, "planes per block in [1, 64]");
        p.kz = v;
        break;
      case FWD_OPT_TILE_ORDER:
        if (v != 0 && v != 1) fail(FWD_ERR_INVALID_ARG, "tile order in {0, 1}");
        p.order = v;
        break;
      case FWD_OPT_VECTOR_H:
        if (v != 1 && v != 4) fail(FWD_ERR_INVALID_ARG, "vector option in {1, 4}");
        if (v != 1 && p.fd_order == 4) fail(FWD_ERR_INVALID_ARG, "order 4 runs with vector 1");
        p.vxh = v;
        break;
      case FWD_OPT_VTI_GRADIENT:
        if (v != 0 && v != 1) fail(FWD_ERR_INVALID_ARG, "VTI gradient option in {0, 1}");
        p.vti_grad = v;
        break;
      case FWD_OPT_FD_ORDER:
        if (v != 2 && v != 4) fail(FWD_ERR_INVALID_ARG, "difference order in {2, 4}");
        if (v != p.fd_order) {
          p.fd_order = v;
          p.have_model = false;          // the tables depend on it: set the model again
          p.have_basis = false;
          ++p.model_version;
        }
        if (v == 4) {
          p.sched = 0;
          p.vx = 1;
          p.vxh = 1;
        }
        break;
      case FWD_OPT_LEAN:
        if (v != 0 && v != 1) fail(FWD_ERR_INVALID_ARG, "lean option in {0, 1}");
        p.lean = v;
        break;
      default:
        fail(FWD_ERR_INVALID_ARG, "unknown option");
    }
  });
}

fwd_status fwd_get_option(const fwd_plan *h, int key, double *value) {
  return guard([&] {
    Plan &p = const_cast<Plan &>(P(h));
    if (!value) fail(FWD_ERR_INVALID_ARG, "value is NULL");
    switch (key) {
      case FWD_OPT_GRAPH_STEPS: *value = p.graph_steps; break;
      case FWD_OPT_BLOCK_X: *value = p.bx; break;
      case FWD_OPT_BLOCK_Y: *value = p.by; break;
      case FWD_OPT_XCD_REMAP: *value = p.xcd; break;
      case FWD_OPT_SAMPLE_EVERY: *value = dev_get_sampling(p); break;
      case FWD_OPT_STRICT_CFL: *value = p.strict_cfl; break;
      case FWD_OPT_DFT_BLOCK: *value = p.kb; break;
      case FWD_OPT_VECTOR: *value = p.vx; break;
      case FWD_OPT_SCHEDULE: *value = p.sched; break;
      case FWD_OPT_ZCHUNK: *value = p.kz; break;
      case FWD_OPT_TILE_ORDER: *value = p.order; break;
      case FWD_OPT_VECTOR_H: *value = p.vxh; break;
      case FWD_OPT_VTI_GRADIENT: *value = p.vti_grad; break;
      case FWD_OPT_FD_ORDER: *value = p.fd_order; break;
      case FWD_OPT_LEAN: *value = p.lean; break;
      case FWD_OPT_BARRIER_US: *value = p.barrier_us; break;
      case FWD_OPT_PERSIST_BLOCKS: *value = p.persist_blocks; break;
      case FWD_OPT_DFT_DECIMATE: *value = p.dec; break;
      case FWD_OPT_BARRIER_SLEEP: *value = p.barrier_sleep; break;
      case FWD_OPT_STREAM_STORES: *value = p.stream_stores; break;
      default: fail(FWD_ERR_INVALID_ARG, "unknown option");
    }
  });
}

fwd_status fwd_autotune(fwd_plan *h, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                        int mode, int steps, double *best_ms, void *stream) {
  return guard([&] {
    Plan &p = P(h);
    if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
    if (!ws) fail(FWD_ERR_INVALID_ARG, "workspace is required");
    if (steps < 1) fail(FWD_ERR_INVALID_ARG, "steps >= 1");
    need_aligned(ws, "workspace");
    need_aligned(vol, "volume buffer");
    const double ms = dev_autotune(p, ws, ws_bytes, vol, vol_bytes, mode, steps, stream);
    if (best_ms) *best_ms = ms;
  });
}

fwd_status fwd_last_timing(const fwd_plan *h, double *ms, int *steps) {
  return guard([&] {
    const Plan &p = P(h);
    if (ms) *ms = p.last_ms;
    if (steps) *steps = p.last_steps;
  });
}

fwd_status fwd_kernel_stats(const fwd_plan *h, double *avg_ms, int *samples) {
  return guard([&] {
    Plan &p = const_cast<Plan &>(P(h));
    if (!avg_ms) fail(FWD_ERR_INVALID_ARG, "avg_ms is NULL");
    int n = 0;
    dev_kernel_stats(p, avg_ms, &n);
    if (samples) *samples = n;
  });
}

}  // extern "C"
