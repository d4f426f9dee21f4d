// Internal declarations of the hyproj library: workspace layout and the
// launch wrappers that the C-ABI entry points call.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hyproj.h"

namespace hyp {

// Device-resident scalars of one projection (lives in the workspace).
struct Scalars {
  double sum_abs_d;   // sum over fluid cells of |d|
  double sum_d2;      // sum over fluid cells of d^2
  double e1_init;     // sum_abs_d / nF
  double s;           // sqrt(sum_d2 / nF): CNN input scale
  double e1_cnn;      // E_1 of the initial guess
  double e1_solve;    // E_1 of the returned iterate as the solver saw it
  double dt;          // time step of the last advection (CFL)
  int32_t nF;         // fluid cells after the pocket fill
  int32_t iters;
  int32_t status;
  int32_t plan_rounds;
  unsigned bar;       // grid-barrier counter (zeroed before each launch)
  unsigned epoch;     // tag epoch of the Jacobi halo words: 0 after planning,
                      // then 1 .. kEpochs, advanced once per projection
  unsigned pad[2];
  double lam_s;       // adjoint of the CNN input scale s
  double loss;        // last backward's loss
};

constexpr int kMaxCoopBlocks = 1024;   // partial-sum slots per parity
constexpr int kMaxCheckpoints = 64;    // Jacobi checkpoint planes per projection
// grid-barrier area: top counter, flag and one counter per group of
// kSyncGroup blocks, each on its own 128-byte line (common.h)
constexpr int kSyncGroup = 16;
constexpr int kSyncSlots = 2 + kMaxCoopBlocks / kSyncGroup;
// the whole area is zeroed before every launch that uses it
constexpr int kSyncBytes = kSyncSlots * 128;
// Tag epochs of the Jacobi halo words (12 bits): at the wrap to 1 the
// kernel clears the words before its first exchange.
constexpr unsigned kEpochs = 4095;
constexpr int kStatusRunning = -1;     // Scalars::status while a solve is in progress
constexpr int kStreamBlock = 256;      // threads of the streaming kernels
constexpr int kStreamGrid = 2048;      // at most this many blocks in the reducing streaming kernels

struct NetShape {
  int scales = 0, channels = 0, precision = 0;
  int arch = 0;        // HYP_ARCH_*
  bool train = false;  // keep every layer's activations for the backward pass
};

constexpr int kWgBlocks = 128;  // pixel-chunk blocks of the weight-gradient reduction

// Byte offsets into the caller's workspace (all 256-byte aligned).
struct WsLayout {
  size_t cell = 0, d = 0, phi = 0, phi_acc = 0, exch = 0, exch64 = 0, blockpart = 0, partial = 0,
         lagflag = 0, scalars = 0, reach = 0, pcg = 0, adv = 0, sync = 0, coef = 0;
  size_t ncell = 0;
  size_t cnn_in = 0, cnn_act0 = 0, cnn_act1 = 0, cnn_y = 0, cnn_t = 0, cnn_w = 0, cnn_cat = 0;
  size_t cnn_save = 0, bw_cells = 0, bw_t = 0, bw_x = 0, bw_a = 0, bw_b = 0, bw_part = 0;
  size_t bw_part_n = 0;
  size_t total = 0;
  size_t blockpart_n = 0;
  int nblocks_stream = 0;
  // per-scale offsets (elements) into the CNN buffers
  int sc_h[6] = {0}, sc_w[6] = {0};
  size_t sc_off_px[6] = {0};  // pixel offset of scale k in the concatenated pyramid
  size_t total_px = 0;
};

WsLayout make_layout(int nx, int ny, const NetShape& net);

// Views of the workspace for one grid.
struct Ws {
  uint8_t* cell;
  float* d;
  float* phi;
  float* phi_acc;     // pressure folded into the faces by defect-correction folds
  float* exch;        // 2 x nx*ny FP32 halo planes (batched kernel; Jacobi tested every step)
  uint64_t* exch64;   // 2 x nx*ny tagged halo words of the Jacobi and PCG kernels
  double* blockpart;  // streaming-kernel block partials
  size_t blockpart_n; // capacity of blockpart in doubles
  double* partial;    // 6 x kMaxCoopBlocks cooperative partials
  unsigned* lagflag;  // 2 x kMaxCoopBlocks tags of the Jacobi kernel's lagged E_1 partials
  Scalars* sc;
  unsigned* sync;     // grid barrier: counter at [0], generation flag at [32]
  uint64_t* reach;   // planner bit words: fluid, then linked (plan_bytes)
  float* pcg;         // PCG scratch
  float* adv;         // advection temporaries: 2 x (cells + u faces + v faces)
  void* cnn_in; void* cnn_act0; void* cnn_act1; float* cnn_y; float* cnn_t; void* cnn_w;
  void* cnn_cat;      // Unet concatenation buffers
  float* coef_e;      // variable-density face coefficients: east face of each cell
  float* coef_n;      // ... north face
  void* cnn_save;     // training: 4 layers x total_px x C activations
  float* bw_cells;    // backward: 3 x cells (lambda ping-pong, lambda_d)
  float* bw_t;        // backward: lambda of t / y, all scales
  float* bw_x;        // backward: lambda of input channel 0, all scales
  float* bw_a;        // backward: activation lambdas (total_px x C) x 2
  float* bw_b;
  float* bw_part;     // backward: weight-gradient partials
  size_t bw_part_n;
};
Ws ws_view(void* base, const WsLayout& L);

struct Device {
  int cu = 256;           // compute units
  int max_lds = 65536;    // LDS bytes per work-group
};

// ---- launch wrappers (return hipSuccess or the first error) ----
size_t plan_bytes(int nx, int ny);
hipError_t run_plan(const Device& dev, int nx, int ny, const uint8_t* flags, const Ws& w,
                    hipStream_t s);
hipError_t run_div(int nx, int ny, double dx, float* u, float* v, const Ws& w,
                   int nblocks, hipStream_t s);
hipError_t run_init_phi(int nx, int ny, const float* p_init, double scale, const Ws& w,
                        hipStream_t s);
hipError_t run_jacobi(const Device& dev, int nx, int ny, double dx, double thr, float omega,
                      int max_iters, int check_every, int fixed_iters, int fold_window,
                      int checkpoint_every, float* phi_ckpt, int tile_rows, int block, bool var,
                      bool einf,
                      float* u, float* v, const Ws& w, hipStream_t s);
bool solver_fits(const Device& dev, int nx, int ny, bool pcg, int check_every, int fixed_iters,
                 int tile_rows, int block, bool var);
hipError_t run_pcg(const Device& dev, int nx, int ny, double dx, double thr, int max_iters,
                   int check_every, int fixed_iters, bool var, bool einf, float* u, float* v,
                   const Ws& w, hipStream_t s);
hipError_t run_grad_and_finish(int nx, int ny, double dx, double rho0, double dt, bool dt_dev,
                               float* u, float* v, float* p, const Ws& w, int nblocks, void* res,
                               bool var, hipStream_t s);
hipError_t run_coef(int nx, int ny, double rho0, const float* rho, const Ws& w, hipStream_t s);
hipError_t run_advect(int nx, int ny, double dx, double g, double rho0, double drho, double u_in,
                      double cfl, float* rho, float* u, float* v, const float* xi, const Ws& w,
                      hipStream_t s);
hipError_t run_backward(const NetShape& net, const WsLayout& L, int nx, int ny, double dx,
                        int sweeps, float omega, double scale, bool accumulate,
                        const float* params, float* du, float* dv, float* dparams,
                        double* loss_out, const Ws& w, hipStream_t s);
hipError_t run_adam(float* params, const float* grads, float* m, float* v, int64_t n, int step,
                    float lr, float b1, float b2, float eps, hipStream_t s);
size_t cnn_weight_image_bytes(const NetShape& net);
int64_t pn_param_count(int arch);
size_t pn_weight_image_bytes(const NetShape& net);
size_t unet_cat_elems(int nx, int ny);
hipError_t run_papernet(const Device& dev, const NetShape& net, const WsLayout& L, int nx, int ny,
                        double dx, const float* params, const Ws& w, hipStream_t s);
hipError_t run_cnn(const Device& dev, const NetShape& net, const WsLayout& L, int nx, int ny,
                   double dx, const float* params, const Ws& w, hipStream_t s);

// hyp_project with all of its checks first, then (plan_first) the planner
// on f->flags ahead of the projection (the no-allocation entry point).
int project_checked(hyp_ctx* ctx, const hyp_grid* g, const hyp_fields* f, double threshold,
                    const hyp_opts* o, void* ws, size_t ws_bytes, hipStream_t stream,
                    hyp_result* res, bool plan_first);

}  // namespace hyp
