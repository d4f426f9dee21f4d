// C-ABI entry points of hyproj: context, workspace layout, planning and the
// projection pipeline (boundary faces + divergence, initial guess, solver,
// gradient correction).  Host code only; every step of the projection runs
// in the kernels of stencil.hip, solvers.hip and cnn.hip.
#include <new>
#include <string.h>
#include <vector>

#include "../../include/hyproj.h"
#include "batch.h"
#include "internal.h"
#include "cascade.h"
#include "unet.h"

struct hyp_ctx {
  hyp::NetShape net;
  hyp::Device dev;
  const float* params = nullptr;
  int64_t n_params_set = 0;
  // phase timing: events recorded on the caller's stream around advection,
  // divergence + CNN, the solver launch, and the correction
  bool timing = false;
  bool timed_step = false;
  bool last_var = false;  // the last forward used the variable-density operator
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

static void mark(hyp_ctx* ctx, int i, hipStream_t s) {
  if (ctx->timing) (void)hipEventRecord(ctx->ev[i], s);
}

namespace hyp {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t cnn_param_count(int S, int C) {
  return (int64_t)S * ((int64_t)C * 9 * 2 + C + 3 * ((int64_t)C * 9 * C + C) + C + 1);
}

WsLayout make_layout(int nx, int ny, const NetShape& net) {
  WsLayout L;
  const size_t n = (size_t)nx * ny;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
  L.nblocks_stream = (int)((n + kStreamBlock - 1) / kStreamBlock);
  L.scalars = take(sizeof(Scalars));
  L.sync = take(kSyncBytes);
  L.partial = take(sizeof(double) * 6 * kMaxCoopBlocks);
  L.lagflag = take(sizeof(unsigned) * 2 * kMaxCoopBlocks);
  // block partials: two per cell-grid block, or one per face-grid block (CFL)
  const size_t nfaces = (size_t)ny * (nx + 1) + (size_t)(ny + 1) * nx;
  const size_t nb_faces = (nfaces + kStreamBlock - 1) / kStreamBlock;
  const size_t nbp = 2 * (size_t)L.nblocks_stream > nb_faces ? 2 * (size_t)L.nblocks_stream : nb_faces;
  L.blockpart = take(sizeof(double) * nbp);
  L.blockpart_n = nbp;
  L.cell = take(n);
  L.reach = take(plan_bytes(nx, ny));
  L.d = take(4 * n);
  L.phi = take(4 * n);
  L.phi_acc = take(4 * n);
  L.exch = take(8 * n);
  L.exch64 = take(16 * n);
  L.coef = take(8 * n);
  L.ncell = n;
  L.adv = take(4 * 2 * (n + (size_t)ny * (nx + 1) + (size_t)(ny + 1) * nx));
  if (net.scales > 0) {
    size_t px = 0;
    for (int k = 0; k < net.scales; ++k) {
      L.sc_h[k] = ny >> k;
      L.sc_w[k] = nx >> k;
      L.sc_off_px[k] = px;
      px += (size_t)L.sc_h[k] * L.sc_w[k];
    }
    L.total_px = px;
    const size_t act_elt = net.precision == HYP_PREC_BF16 ? 2 : 4;
    // the cascaded networks feed 3 input channels to the finest branch
    L.cnn_in = take((net.arch == HYP_ARCH_PARALLEL ? px * 2 : n * 3) * act_elt);
    L.cnn_act0 = take(px * net.channels * act_elt);
    L.cnn_act1 = take(px * net.channels * act_elt);
    L.cnn_y = take(px * 4);
    L.cnn_t = take(px * 4);
    L.cnn_w = take(cnn_weight_image_bytes(net));
    if (net.arch == HYP_ARCH_UNET) L.cnn_cat = take(unet_cat_elems(nx, ny) * act_elt);
    if (net.train && (net.arch == HYP_ARCH_MULTISCALE || net.arch == HYP_ARCH_SMALLSCALE)) {
      // every branch input and layer output (cascade.h); lambda maps of up
      // to C channels at full resolution; the branches' input lambdas (2-3
      // channels) go to bw_b
      const size_t C = net.channels;
      L.cnn_save = take(4 * pn_save_layout(net.arch, nx, ny).total);
      L.bw_cells = take(3 * 4 * n);
      L.bw_t = take(4 * px);
      L.bw_x = take(4 * px);
      L.bw_a = take(4 * n * C);
      L.bw_b = take(4 * n * C);
      L.bw_part_n = (size_t)kWgBlocks * (C * 9 * C + C);
      L.bw_part = take(4 * L.bw_part_n);
    } else if (net.train && net.arch == HYP_ARCH_UNET) {
      // every layer's FP32 output and the skip gradients (unet.h); lambda
      // maps of up to 32 channels at full resolution (the concatenation)
      const size_t C = net.channels;
      L.cnn_save = take(4 * unet_save_layout(nx, ny).total);
      L.bw_cells = take(3 * 4 * n);
      L.bw_t = take(4 * px);
      L.bw_x = take(4 * px);
      L.bw_a = take(4 * px * C);
      L.bw_b = take(4 * px * C);
      L.bw_part_n = (size_t)kWgBlocks * (C * 9 * C + C);
      L.bw_part = take(4 * L.bw_part_n);
    } else if (net.train) {
      const size_t C = net.channels;
      L.cnn_save = take(4 * px * C * act_elt);
      L.bw_cells = take(3 * 4 * n);
      L.bw_t = take(4 * px);
      L.bw_x = take(4 * px);
      L.bw_a = take(4 * px * C);
      L.bw_b = take(4 * px * C);
      L.bw_part_n = (size_t)kWgBlocks * (C * 9 * C + C);
      L.bw_part = take(4 * L.bw_part_n);
    }
  }
  L.total = o;
  return L;
}

Ws ws_view(void* base, const WsLayout& L) {
  char* b = (char*)base;
  Ws w;
  w.sc = (Scalars*)(b + L.scalars);
  w.sync = (unsigned*)(b + L.sync);
  w.partial = (double*)(b + L.partial);
  w.lagflag = (unsigned*)(b + L.lagflag);
  w.blockpart = (double*)(b + L.blockpart);
  w.blockpart_n = L.blockpart_n;
  w.cell = (uint8_t*)(b + L.cell);
  w.reach = (uint64_t*)(b + L.reach);
  w.d = (float*)(b + L.d);
  w.phi = (float*)(b + L.phi);
  w.phi_acc = (float*)(b + L.phi_acc);
  w.exch = (float*)(b + L.exch);
  w.exch64 = (uint64_t*)(b + L.exch64);
  w.coef_e = (float*)(b + L.coef);
  w.coef_n = w.coef_e + L.ncell;
  w.pcg = nullptr;
  w.adv = (float*)(b + L.adv);
  w.cnn_in = L.cnn_in ? b + L.cnn_in : nullptr;
  w.cnn_act0 = L.cnn_act0 ? b + L.cnn_act0 : nullptr;
  w.cnn_act1 = L.cnn_act1 ? b + L.cnn_act1 : nullptr;
  w.cnn_y = L.cnn_y ? (float*)(b + L.cnn_y) : nullptr;
  w.cnn_t = L.cnn_t ? (float*)(b + L.cnn_t) : nullptr;
  w.cnn_w = L.cnn_w ? b + L.cnn_w : nullptr;
  w.cnn_cat = L.cnn_cat ? b + L.cnn_cat : nullptr;
  w.cnn_save = L.cnn_save ? b + L.cnn_save : nullptr;
  w.bw_cells = L.bw_cells ? (float*)(b + L.bw_cells) : nullptr;
  w.bw_t = L.bw_t ? (float*)(b + L.bw_t) : nullptr;
  w.bw_x = L.bw_x ? (float*)(b + L.bw_x) : nullptr;
  w.bw_a = L.bw_a ? (float*)(b + L.bw_a) : nullptr;
  w.bw_b = L.bw_b ? (float*)(b + L.bw_b) : nullptr;
  w.bw_part = L.bw_part ? (float*)(b + L.bw_part) : nullptr;
  w.bw_part_n = L.bw_part_n;
  return w;
}

}  // namespace hyp

using namespace hyp;

static int grid_ok(const hyp_grid* g) {
  if (!g) return 0;
  if (g->nx < 2 || g->ny < 2 || g->nx > 16384 || g->ny > 16384) return 0;
  if ((int64_t)g->nx * g->ny > (int64_t)1 << 28) return 0;
  if (!(g->dx > 0.0) || !(g->dt > 0.0) || !(g->rho0 > 0.0)) return 0;
  return 1;
}

extern "C" {

int hyp_version(void) { return HYP_VERSION; }

const char* hyp_status_str(int code) {
  switch (code) {
    case HYP_OK: return "ok";
    case HYP_EINVAL: return "invalid argument";
    case HYP_EUNSUPPORTED: return "unsupported shape or option";
    case HYP_EWORKSPACE: return "workspace too small";
    case HYP_EHIP: return "HIP error";
    case HYP_EINTERNAL: return "internal error";
    case HYP_ENOWEIGHTS: return "CNN method without network weights";
    default: return "unknown";
  }
}

int hyp_create(hyp_ctx** out, const hyp_net_desc* net) {
  if (!out) return HYP_EINVAL;
  *out = nullptr;
  NetShape ns;
  if (net && (net->arch == HYP_ARCH_MULTISCALE || net->arch == HYP_ARCH_SMALLSCALE ||
              net->arch == HYP_ARCH_UNET)) {
    // the paper's networks: fixed scales and widths
    const int S = net->arch == HYP_ARCH_UNET ? 5 : 3;
    const int C = net->arch == HYP_ARCH_SMALLSCALE ? 32 : 64;
    if ((net->scales != 0 && net->scales != S) || (net->channels != 0 && net->channels != C))
      return HYP_EINVAL;
    if (net->precision != HYP_PREC_FP32 && net->precision != HYP_PREC_BF16) return HYP_EINVAL;
    if (net->flags & ~HYP_NET_TRAIN) return HYP_EINVAL;
    // training: FP32 only
    if ((net->flags & HYP_NET_TRAIN) && net->precision != HYP_PREC_FP32) return HYP_EUNSUPPORTED;
    ns.scales = S;
    ns.channels = C;
    ns.precision = net->precision;
    ns.arch = net->arch;
    ns.train = (net->flags & HYP_NET_TRAIN) != 0;
  } else if (net) {
    if (net->arch != HYP_ARCH_PARALLEL) return HYP_EINVAL;
    if (net->scales < 1 || net->scales > 5) return HYP_EINVAL;
    if (net->precision == HYP_PREC_FP32) {
      if (net->channels != 16 && net->channels != 32 && net->channels != 64) return HYP_EINVAL;
      // the FP32 64-channel network is inference only
      if (net->channels == 64 && (net->flags & HYP_NET_TRAIN)) return HYP_EUNSUPPORTED;
    } else if (net->precision == HYP_PREC_BF16) {
      if (net->channels != 32 && net->channels != 64) return HYP_EINVAL;
    } else {
      return HYP_EINVAL;
    }
    if (net->flags & ~HYP_NET_TRAIN) return HYP_EINVAL;
    ns.scales = net->scales;
    ns.channels = net->channels;
    ns.precision = net->precision;
    ns.train = (net->flags & HYP_NET_TRAIN) != 0;
  }
  hyp_ctx* c = new (std::nothrow) hyp_ctx;
  if (!c) return HYP_EINTERNAL;
  c->net = ns;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int cu = 0, lds = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      c->dev.cu = cu;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        lds > 0)
      c->dev.max_lds = lds;
  }
  *out = c;
  return HYP_OK;
}

int hyp_destroy(hyp_ctx* ctx) {
  if (!ctx) return HYP_OK;
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return HYP_OK;
}

int hyp_set_timing(hyp_ctx* ctx, int enable) {
  if (!ctx) return HYP_EINVAL;
  if (enable && !ctx->ev[0]) {
    for (auto& e : ctx->ev)
      if (hipEventCreate(&e) != hipSuccess) return HYP_EHIP;
  }
  ctx->timing = enable != 0;
  return HYP_OK;
}

int hyp_get_timing(hyp_ctx* ctx, float* ms) {
  if (!ctx || !ms) return HYP_EINVAL;
  if (!ctx->timing) return HYP_EINVAL;
  for (int i = 0; i < 5; ++i) ms[i] = 0.f;
  for (int i = 0; i < 5; ++i)
    if (hipEventSynchronize(ctx->ev[i]) != hipSuccess) return HYP_EHIP;
  float t = 0.f;
  if (ctx->timed_step && hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]) == hipSuccess) ms[0] = t;
  if (hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]) == hipSuccess) ms[1] = t;
  if (hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]) == hipSuccess) ms[2] = t;
  if (hipEventElapsedTime(&t, ctx->ev[3], ctx->ev[4]) == hipSuccess) ms[3] = t;
  if (hipEventElapsedTime(&t, ctx->timed_step ? ctx->ev[0] : ctx->ev[1], ctx->ev[4]) == hipSuccess)
    ms[4] = t;
  return HYP_OK;
}

int64_t hyp_param_count(const hyp_ctx* ctx) {
  if (!ctx || ctx->net.scales == 0) return 0;
  if (ctx->net.arch != HYP_ARCH_PARALLEL) return pn_param_count(ctx->net.arch);
  return cnn_param_count(ctx->net.scales, ctx->net.channels);
}

int hyp_set_weights(hyp_ctx* ctx, const float* dev_params, int64_t n_params) {
  if (!ctx || !dev_params) return HYP_EINVAL;
  if (ctx->net.scales == 0) return HYP_ENOWEIGHTS;
  if (n_params != hyp_param_count(ctx)) return HYP_EINVAL;
  ctx->params = dev_params;
  ctx->n_params_set = n_params;
  return HYP_OK;
}

int hyp_workspace_size(const hyp_ctx* ctx, const hyp_grid* g, size_t* bytes) {
  if (!ctx || !bytes || !grid_ok(g)) return HYP_EINVAL;
  *bytes = make_layout(g->nx, g->ny, ctx->net).total;
  return HYP_OK;
}

int hyp_plan(hyp_ctx* ctx, const hyp_grid* g, const uint8_t* flags, void* ws, size_t ws_bytes,
             hipStream_t stream) {
  if (!ctx || !flags || !ws || !grid_ok(g)) return HYP_EINVAL;
  const WsLayout L = make_layout(g->nx, g->ny, ctx->net);
  if (ws_bytes < L.total) return HYP_EWORKSPACE;
  const Ws w = ws_view(ws, L);
  if (run_plan(ctx->dev, g->nx, g->ny, flags, w, stream) != hipSuccess) return HYP_EHIP;
  return HYP_OK;
}

static int check_opts(const hyp_ctx* ctx, const hyp_grid* g, const hyp_opts* o, double threshold) {
  if (o->method < HYP_METHOD_HYBRID || o->method > HYP_METHOD_CNN) return HYP_EINVAL;
  if (o->max_iters < 0 || o->check_every < 1 || o->fixed_iters < 0) return HYP_EINVAL;
  if (o->fold_window < 0 || o->checkpoint_every < 0) return HYP_EINVAL;
  if (!(o->omega > 0.f)) return HYP_EINVAL;
  if (o->variable_density != 0 && o->variable_density != 1) return HYP_EINVAL;
  if (o->criterion != HYP_CRIT_E1 && o->criterion != HYP_CRIT_EINF) return HYP_EINVAL;
  if (!(threshold >= 0.0)) return HYP_EINVAL;
  const bool use_cnn = o->method == HYP_METHOD_HYBRID || o->method == HYP_METHOD_CNN;
  if (use_cnn) {
    if (ctx->net.scales == 0 || !ctx->params) return HYP_ENOWEIGHTS;
    const int m = 1 << (ctx->net.scales - 1);
    if (g->nx % m || g->ny % m) return HYP_EUNSUPPORTED;
  }
  const bool pcg = o->method == HYP_METHOD_PCG;
  if (o->tile_rows < 0 || (pcg && o->tile_rows != 0)) return HYP_EINVAL;
  if (o->block_sweeps < 0 || o->block_sweeps > 16 || (pcg && o->block_sweeps != 0)) return HYP_EINVAL;
  if (!solver_fits(ctx->dev, g->nx, g->ny, pcg, o->check_every, o->fixed_iters, o->tile_rows,
                   o->block_sweeps, o->variable_density != 0))
    return HYP_EUNSUPPORTED;
  return HYP_OK;
}

// The projection pipeline, enqueued on `stream` (arguments already checked).
static int enqueue_projection(hyp_ctx* ctx, const hyp_grid* g, float* u, float* v,
                              const float* rho, const float* p_init, float* p, float* phi_ckpt,
                              double threshold, const hyp_opts* o,
                              const WsLayout& L, const Ws& w, bool dt_dev, hipStream_t stream,
                              hyp_result* res) {
  const int nx = g->nx, ny = g->ny;
  const bool use_cnn = o->method == HYP_METHOD_HYBRID || o->method == HYP_METHOD_CNN;
  const bool var = o->variable_density != 0;
  const bool einf = o->criterion == HYP_CRIT_EINF;
  ctx->last_var = var;
  mark(ctx, 1, stream);
  if (run_div(nx, ny, g->dx, u, v, w, L.nblocks_stream, stream) != hipSuccess) return HYP_EHIP;
  if (var && run_coef(nx, ny, g->rho0, rho, w, stream) != hipSuccess) return HYP_EHIP;
  if (use_cnn) {
    if (run_cnn(ctx->dev, ctx->net, L, nx, ny, g->dx, ctx->params, w, stream) != hipSuccess)
      return HYP_EHIP;
  } else {
    if (run_init_phi(nx, ny, p_init, g->dt / g->rho0, w, stream) != hipSuccess) return HYP_EHIP;
  }
  hipError_t e = hipSuccess;
  mark(ctx, 2, stream);
  if (o->method == HYP_METHOD_CNN) {
    // no sweeps: a zero-length Jacobi pass records E_1 of the prediction
    e = run_jacobi(ctx->dev, nx, ny, g->dx, HUGE_VAL, 1.0f, 0, 1, 0, 0, 0, nullptr, 0, 0, var, einf, u,
                   v, w, stream);
  } else if (o->method == HYP_METHOD_PCG) {
    // one persistent launch, defect-correction folds included
    e = run_pcg(ctx->dev, nx, ny, g->dx, threshold, o->max_iters, o->check_every,
                o->fixed_iters, var, einf, u, v, w, stream);
  } else {
    // one persistent launch, defect-correction folds included
    e = run_jacobi(ctx->dev, nx, ny, g->dx, threshold, o->omega, o->max_iters, o->check_every,
                   o->fixed_iters, o->fold_window, phi_ckpt ? o->checkpoint_every : 0, phi_ckpt,
                   o->tile_rows, o->block_sweeps, var, einf, u, v, w, stream);
  }
  if (e != hipSuccess) return HYP_EHIP;
  mark(ctx, 3, stream);
  if (run_grad_and_finish(nx, ny, g->dx, g->rho0, g->dt, dt_dev, u, v, p, w, L.nblocks_stream,
                          res, var, stream) != hipSuccess)
    return HYP_EHIP;
  mark(ctx, 4, stream);
  return HYP_OK;
}

int hyp_project(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f, double threshold,
                const hyp_opts* o, void* ws, size_t ws_bytes, hipStream_t stream,
                hyp_result* res) {
  return hyp::project_checked(ctx, g, f, threshold, o, ws, ws_bytes, stream, res, false);
}

}  // extern "C"

// hyp_project's checks, then (plan_first) the planner on f->flags and the
// projection: every argument is validated before anything is enqueued.
int hyp::project_checked(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f, double threshold,
                         const hyp_opts* o, void* ws, size_t ws_bytes, hipStream_t stream,
                         hyp_result* res, bool plan_first) {
  if (!ctx || !f || !o || !ws || !res || !grid_ok(g)) return HYP_EINVAL;
  if (!f->u || !f->v || !f->flags || !f->p) return HYP_EINVAL;
  int rc = check_opts(ctx, g, o, threshold);
  if (rc != HYP_OK) return rc;
  if (o->checkpoint_every > 0) {
    if (o->fixed_iters <= 0 || !f->phi_ckpt) return HYP_EINVAL;
    if (o->method != HYP_METHOD_HYBRID && o->method != HYP_METHOD_JACOBI) return HYP_EINVAL;
    if (o->fixed_iters / o->checkpoint_every > kMaxCheckpoints) return HYP_EINVAL;
  }
  const WsLayout L = make_layout(g->nx, g->ny, ctx->net);
  if (ws_bytes < L.total) return HYP_EWORKSPACE;
  const Ws w = ws_view(ws, L);
  if (o->variable_density && !f->rho) return HYP_EINVAL;
  if (plan_first && run_plan(ctx->dev, g->nx, g->ny, f->flags, w, stream) != hipSuccess)
    return HYP_EHIP;
  ctx->timed_step = false;
  return enqueue_projection(ctx, g, f->u, f->v, f->rho, f->p_init, f->p,
                            o->checkpoint_every > 0 ? f->phi_ckpt : nullptr, threshold, o, L, w,
                            false, stream, res);
}

extern "C" {

int hyp_project_backward(hyp_ctx* ctx, const hyp_grid* g, int32_t sweeps, float omega,
                         double scale, int32_t accumulate, float* du, float* dv, float* dparams,
                         double* loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx || !ws || !grid_ok(g) || sweeps < 0) return HYP_EINVAL;
  if (ctx->net.scales == 0 || !ctx->params) return HYP_ENOWEIGHTS;
  if (!ctx->net.train) return HYP_EUNSUPPORTED;
  if (ctx->last_var) return HYP_EUNSUPPORTED;  // the adjoint is of the constant-coefficient projection
  const WsLayout L = make_layout(g->nx, g->ny, ctx->net);
  if (ws_bytes < L.total) return HYP_EWORKSPACE;
  const Ws w = ws_view(ws, L);
  if (run_backward(ctx->net, L, g->nx, g->ny, g->dx, sweeps, omega, scale, accumulate != 0,
                   ctx->params, du, dv, dparams, loss, w, stream) != hipSuccess)
    return HYP_EHIP;
  return HYP_OK;
}

int hyp_adam(float* params, const float* grads, float* m, float* v, int64_t n, int32_t step,
             float lr, float beta1, float beta2, float eps, hipStream_t stream) {
  if (!params || !grads || !m || !v || n <= 0 || step < 1) return HYP_EINVAL;
  if (run_adam(params, grads, m, v, n, step, lr, beta1, beta2, eps, stream) != hipSuccess)
    return HYP_EHIP;
  return HYP_OK;
}

int hyp_advect(hyp_ctx* ctx, const hyp_grid* g, const hyp_physics* ph, const hyp_state* st,
               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx || !ph || !st || !ws) return HYP_EINVAL;
  if (!g || g->nx < 2 || g->ny < 2 || !(g->dx > 0.0) || !(g->rho0 > 0.0)) return HYP_EINVAL;
  if (!st->rho || !st->u || !st->v || !st->xi) return HYP_EINVAL;
  if (!(ph->cfl > 0.0) || !(ph->u_in > 0.0) || !(ph->rho0 > 0.0)) return HYP_EINVAL;
  const WsLayout L = make_layout(g->nx, g->ny, ctx->net);
  if (ws_bytes < L.total) return HYP_EWORKSPACE;
  const Ws w = ws_view(ws, L);
  if (run_advect(g->nx, g->ny, g->dx, ph->g, ph->rho0, ph->drho, ph->u_in, ph->cfl, st->rho, st->u,
                 st->v, st->xi, w, stream) != hipSuccess)
    return HYP_EHIP;
  return HYP_OK;
}

int hyp_step(hyp_ctx* ctx, const hyp_grid* g, const hyp_physics* ph, const hyp_state* st,
             double threshold, const hyp_opts* o, void* ws, size_t ws_bytes, hipStream_t stream,
             hyp_result* res) {
  if (!ctx || !ph || !st || !o || !ws || !res) return HYP_EINVAL;
  if (!g || g->nx < 2 || g->ny < 2 || !(g->dx > 0.0) || !(g->rho0 > 0.0)) return HYP_EINVAL;
  if (!st->rho || !st->u || !st->v || !st->p || !st->flags || !st->xi) return HYP_EINVAL;
  if (!(ph->cfl > 0.0) || !(ph->u_in > 0.0) || !(ph->rho0 > 0.0)) return HYP_EINVAL;
  hyp_grid gg = *g;
  gg.dt = 1.0;  // placeholder for the checks; the pressure uses the device dt
  if (!grid_ok(&gg)) return HYP_EINVAL;
  int rc = check_opts(ctx, &gg, o, threshold);
  if (rc != HYP_OK) return rc;
  if (o->checkpoint_every != 0) return HYP_EINVAL;
  const WsLayout L = make_layout(g->nx, g->ny, ctx->net);
  if (ws_bytes < L.total) return HYP_EWORKSPACE;
  const Ws w = ws_view(ws, L);
  ctx->timed_step = true;
  mark(ctx, 0, stream);
  if (run_advect(g->nx, g->ny, g->dx, ph->g, ph->rho0, ph->drho, ph->u_in, ph->cfl, st->rho, st->u,
                 st->v, st->xi, w, stream) != hipSuccess)
    return HYP_EHIP;
  return enqueue_projection(ctx, &gg, st->u, st->v, st->rho, nullptr, st->p, nullptr, threshold, o, L,
                            w, true, stream, res);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched projection of many plumes of uneven sizes: per phase one launch
// over every instance (batch.h), the Jacobi sweeps in one persistent launch.
struct hyp_batch {
  hyp_ctx* ctx = nullptr;
  int n = 0, ntiles = 0, ntiles_max = 0;
  size_t cnn_bytes = 0;
  int cnn_tiles[4] = {0, 0, 0, 0};
  int tile_mode = 0;  // tile variants of the persistent Jacobi launch
  int test_passes = 1, max_iters = 0;  // E_1 test interval in passes of 8 sweeps
  bool cnn = false, var = false, physics = false;
  std::vector<WsLayout> layouts;
  std::vector<Ws> ws;
  void* area = nullptr;
  hyp::BatchDevice dev{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Batch area, then one projection workspace per instance; the tile count is
// bounded by the smallest tiles (R = 8) so that the size does not depend on
// the options.
static size_t batch_layout(hyp_ctx* ctx, int n, const hyp_grid* grids, std::vector<size_t>* offs,
                           int* ntiles_max, size_t* cnn_bytes) {
  int nt = 0;
  for (int i = 0; i < n; ++i) nt += batch_tiles_of(grids[i].nx, grids[i].ny, 8);
  const size_t cb = ctx->net.scales > 0 && ctx->net.arch == HYP_ARCH_PARALLEL
                        ? cnn_batch_bytes(ctx->net, n) : 0;
  size_t o = align256(batch_area_bytes(n, nt, cb));
  for (int i = 0; i < n; ++i) {
    if (offs) offs->push_back(o);
    o = align256(o + make_layout(grids[i].nx, grids[i].ny, ctx->net).total);
  }
  if (ntiles_max) *ntiles_max = nt;
  if (cnn_bytes) *cnn_bytes = cb;
  return o;
}

extern "C" {

int hyp_batch_workspace_size(hyp_ctx* ctx, int32_t n, const hyp_grid* grids, size_t* bytes) {
  if (!ctx || n < 1 || !grids || !bytes) return HYP_EINVAL;
  for (int i = 0; i < n; ++i) {
    hyp_grid g = grids[i];
    g.dt = g.dt > 0.0 ? g.dt : 1.0;
    if (!grid_ok(&g)) return HYP_EINVAL;
  }
  *bytes = batch_layout(ctx, n, grids, nullptr, nullptr, nullptr);
  return HYP_OK;
}

int hyp_batch_create(hyp_ctx* ctx, int32_t n, const hyp_grid* grids, const hyp_state* states,
                     const double* thresholds, const hyp_physics* physics, const hyp_opts* o,
                     void* ws, size_t ws_bytes, hyp_batch** out) {
  if (!ctx || n < 1 || !grids || !states || !thresholds || !o || !ws || !out) return HYP_EINVAL;
  *out = nullptr;
  if (o->method != HYP_METHOD_HYBRID && o->method != HYP_METHOD_JACOBI) return HYP_EUNSUPPORTED;
  if (o->criterion != HYP_CRIT_E1) return HYP_EUNSUPPORTED;
  if (o->variable_density != 0 && o->variable_density != 1) return HYP_EINVAL;
  if (o->max_iters < 0 || !(o->omega > 0.f) || o->checkpoint_every != 0) return HYP_EINVAL;
  if (o->check_every < 1) return HYP_EINVAL;
  if (o->tile_rows != 0 && o->tile_rows != 8 && o->tile_rows != 16) return HYP_EINVAL;
  if (o->block_sweeps != 0) return HYP_EINVAL;  // the batch sweeps 8 per exchange
  const bool cnn = o->method == HYP_METHOD_HYBRID;
  if (cnn && (ctx->net.scales == 0 || !ctx->params)) return HYP_ENOWEIGHTS;
  if (cnn && (ctx->net.arch != HYP_ARCH_PARALLEL || ctx->net.scales > kBatchMaxScales))
    return HYP_EUNSUPPORTED;
  const bool var = o->variable_density != 0;
  for (int i = 0; i < n; ++i) {
    hyp_grid g = grids[i];
    g.dt = g.dt > 0.0 ? g.dt : 1.0;
    if (!grid_ok(&g) || !(thresholds[i] >= 0.0)) return HYP_EINVAL;
    const hyp_state& st = states[i];
    if (!st.u || !st.v || !st.p || !st.flags) return HYP_EINVAL;
    if (var && !st.rho) return HYP_EINVAL;
    if (physics) {
      const hyp_physics& ph = physics[i];
      if (!(ph.cfl > 0.0) || !(ph.u_in > 0.0) || !(ph.rho0 > 0.0)) return HYP_EINVAL;
    }
    if (cnn) {
      const int m = 1 << (ctx->net.scales - 1);
      if (g.nx % m || g.ny % m) return HYP_EUNSUPPORTED;
    }
  }
  std::vector<size_t> offs;
  int ntiles_max = 0;
  size_t cnn_bytes = 0;
  const size_t need = batch_layout(ctx, n, grids, &offs, &ntiles_max, &cnn_bytes);
  if (ws_bytes < need) return HYP_EWORKSPACE;
  hyp_batch* b = new (std::nothrow) hyp_batch;
  if (!b) return HYP_EINTERNAL;
  b->ctx = ctx;
  b->n = n;
  b->ntiles_max = ntiles_max;
  b->cnn_bytes = cnn_bytes;
  b->cnn = cnn;
  b->var = var;
  b->physics = physics != nullptr;
  b->area = ws;
  b->test_passes = (o->check_every + kBatchSweeps - 1) / kBatchSweeps;
  b->max_iters = o->max_iters;
  std::vector<BInst> binst(n);
  std::vector<int> rows(n);
  int ntiles = 0;
  for (int i = 0; i < n; ++i) {
    const hyp_grid& g = grids[i];
    const hyp_state& st = states[i];
    b->layouts.push_back(make_layout(g.nx, g.ny, ctx->net));
    b->ws.push_back(ws_view((char*)ws + offs[i], b->layouts.back()));
    const WsLayout& Ly = b->layouts.back();
    BInst& B = binst[i];
    B = BInst{};
    B.nx = g.nx; B.ny = g.ny; B.dx = g.dx; B.rho0 = g.rho0;
    B.dt = g.dt > 0.0 ? g.dt : 1.0;
    if (physics) {
      B.g = physics[i].g; B.drho = physics[i].drho; B.u_in = physics[i].u_in;
      B.cfl = physics[i].cfl;
    }
    B.var = var ? 1 : 0;
    B.S = cnn ? ctx->net.scales : 0;
    B.u = st.u; B.v = st.v; B.rho = st.rho; B.p = st.p; B.xi = st.xi; B.flags = st.flags;
    B.w = b->ws.back();
    for (int k = 0; k < B.S; ++k) {
      B.sc_h[k] = Ly.sc_h[k];
      B.sc_w[k] = Ly.sc_w[k];
      B.sc_off_px[k] = Ly.sc_off_px[k];
    }
    rows[i] = batch_rows_of(g.nx, g.ny, var, o->tile_rows);
    ntiles += batch_tiles_of(g.nx, g.ny, rows[i]);
  }
  b->ntiles = ntiles;
  b->tile_mode = batch_tile_mode(n, rows.data(), var);
  // the tables sit at the front of the area, sized for ntiles_max tiles
  const BatchDevice probe = batch_device(ws, n, ntiles, cnn_bytes);
  for (int i = 0; i < n; ++i) binst[i].res = probe.results + i;
  std::vector<double> thr(thresholds, thresholds + n);
  if (batch_setup(ws, n, ntiles, cnn_bytes, binst.data(), rows.data(), thr.data(), o->max_iters,
                  o->omega, &b->dev) != hipSuccess) {
    delete b;
    return HYP_EHIP;
  }
  if (cnn && cnn_batch_setup(ctx->net, n, b->layouts.data(), b->ws.data(), ctx->params,
                             b->dev.cnn_tables, b->cnn_tiles) != hipSuccess) {
    delete b;
    return HYP_EHIP;
  }
  for (int i = 0; i < n; ++i)
    if (run_plan(ctx->dev, grids[i].nx, grids[i].ny, states[i].flags, b->ws[i], nullptr) != hipSuccess) {
      delete b;
      return HYP_EHIP;
    }
  if (hipDeviceSynchronize() != hipSuccess) {
    delete b;
    return HYP_EHIP;
  }
  *out = b;
  return HYP_OK;
}

}  // extern "C"

static int batch_enqueue(hyp_batch* b, bool step, hipStream_t s, hyp_result* res, bool cooperative) {
  hyp_ctx* ctx = b->ctx;
  const BInst* I = b->dev.binst;
  const BatchRanges& R = b->dev.ranges;
  if (step && run_advect_batch(I, R, s) != hipSuccess) return HYP_EHIP;
  if (run_div_batch(I, R, s) != hipSuccess) return HYP_EHIP;
  if (b->var && run_coef_batch(I, R, s) != hipSuccess) return HYP_EHIP;
  if (b->cnn) {
    if (run_cnn_batch(ctx->dev, ctx->net, I, R, b->dev.cnn_tables, b->cnn_tiles, b->ws[0],
                      ctx->params, s) != hipSuccess)
      return HYP_EHIP;
  } else if (run_init_phi_batch(I, R, s) != hipSuccess) {
    return HYP_EHIP;
  }
  if (run_jacobi_batch(ctx->dev, b->area, b->n, b->ntiles, b->cnn_bytes, b->tile_mode,
                       b->test_passes, b->max_iters, cooperative, s) != hipSuccess)
    return HYP_EHIP;
  if (run_grad_finish_batch(I, R, step, b->var, s) != hipSuccess) return HYP_EHIP;
  if (hipMemcpyAsync(res, b->dev.results, sizeof(hyp_result) * b->n, hipMemcpyDefault, s) != hipSuccess)
    return HYP_EHIP;
  return HYP_OK;
}

extern "C" {

int hyp_batch_project(hyp_batch* b, hipStream_t stream, hyp_result* res) {
  if (!b || !res) return HYP_EINVAL;
  return batch_enqueue(b, false, stream, res, true);
}

int hyp_batch_step(hyp_batch* b, hipStream_t stream, hyp_result* res) {
  if (!b || !res) return HYP_EINVAL;
  if (!b->physics) return HYP_EINVAL;
  return batch_enqueue(b, true, stream, res, true);
}

int hyp_batch_capture(hyp_batch* b, hipStream_t stream, hyp_result* res) {
  if (!b || !res || !stream) return HYP_EINVAL;
  if (!b->physics) return HYP_EINVAL;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return HYP_EHIP;
  const int rc = batch_enqueue(b, true, stream, res, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(stream, &g);
  if (rc != HYP_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc != HYP_OK ? rc : HYP_EHIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return HYP_EHIP;
  return HYP_OK;
}

int hyp_batch_launch(hyp_batch* b, hipStream_t stream) {
  if (!b || !b->exec) return HYP_EINVAL;
  return hipGraphLaunch(b->exec, stream) == hipSuccess ? HYP_OK : HYP_EHIP;
}

int hyp_batch_destroy(hyp_batch* b) {
  if (!b) return HYP_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
  return HYP_OK;
}

}  // extern "C"
