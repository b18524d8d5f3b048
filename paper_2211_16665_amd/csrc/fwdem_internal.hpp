// Internal declarations shared by the host setup (setup.cpp), the device
// driver (device.hip) and the C ABI (api.cpp).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "fwdem.h"

namespace fwdem {

using cplx = std::complex<double>;

struct Error {
  fwd_status code;
  std::string msg;
};
[[noreturn]] void fail(fwd_status code, const std::string &msg);

constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kPi = 3.14159265358979323846;

// Defaults of the CPML and of the step count (mirrored by no other code:
// the oracle states the same definitions independently).
constexpr double kCpmlOrder = 2.0;
constexpr double kCpmlR = 1.0e-6;
constexpr double kCpmlKappaMax = 1.0;
constexpr double kCpmlAlphaFactor = 0.5;  // alpha_max = factor * sqrt(omega_min omega0)
constexpr double kNtTol = 1.0e-11;        // exp(-a_min nt dt)
constexpr double kDefaultCap = 1.0e4;
constexpr double kDefaultCfl = 0.95;

struct Axis {
  int n = 0;                     // cells
  std::vector<double> nodes;     // n+1
  std::vector<double> h;         // n   cell widths
  std::vector<double> hd;        // n+1 dual widths (half a cell at the ends)
  // metric lengths dividing the differences: n at the half nodes, n+1 at the
  // nodes (h and hd for order 2; the fourth-order pair applied to the
  // coordinates for order 4)
  std::vector<double> m, md;
  // CPML: 1/kappa, b, a at integer nodes (n+1) and half nodes (n)
  std::vector<double> kinv_n, b_n, a_n;
  std::vector<double> kinv_h, b_h, a_h;
};

// One injection target: component c of source s (0..2: an E edge, 3..5: an H
// node) at linear index idx of the padded device layout; the per-step value is
// sum_r coef[toff + r] * F[r][n] with nrow rows of time functions F.
struct Target {
  int s;
  int c;
  int64_t idx;
  int toff;
};

struct Plan {
  // ---- description ----
  int nx = 0, ny = 0, nz = 0, npml = 0;
  int NX = 0, NY = 0, NZ = 0, PX = 0;   // node counts and padded x pitch
  Axis ax[3];
  double cpml_order = 0, cpml_R = 0, cpml_kmax = 0, cpml_amax_in = 0, cpml_vref_in = 0;
  double f0 = 0, omega0 = 0;
  std::vector<double> freqs, omega, a;   // a = sqrt(omega omega0)
  std::vector<cplx> wprime;              // (1+i) a
  int ns = 0, nr = 0, ncomp = 0;
  int src_kind = 0;                      // 0: electric dipoles (J), 1: magnetic dipoles (M)
  std::vector<double> src_pos, src_mom, rec_pos;
  std::vector<int> comp;
  int dtype = FWD_F32, acc = FWD_ACC_F64;
  double cap = 0, cfl = 0, dt_user = 0;
  int nt_user = 0;

  // ---- derived from the model ----
  bool have_model = false;
  std::vector<double> rho, sigma;        // rho_h and sigma_h in VTI
  std::vector<uint8_t> capped;
  bool vti = false;                      // vertical resistivity given
  std::vector<double> sigma_v;           // = sigma when isotropic
  std::vector<uint8_t> capped_v;
  std::vector<double> sig_e[3];          // edge conductivity, padded layout
  std::vector<double> ce[3];             // dt/eps on updated edges, 0 elsewhere
  double dt = 0, dt_cfl = 0, vmax = 0, vref = 0, amax = 0;
  int nt = 0;
  std::vector<double> wavelet;           // [nt]
  double tau = 0, t0 = 0;
  std::vector<cplx> What, norm, Omega;   // [nf]; What: transform of the injected wavelet
  std::vector<cplx> zE;                  // [nt][nf] z^{n+1}
  std::vector<cplx> zH;                  // [nt][nf] z^{n+1/2} (H samples)
  std::vector<cplx> norm_h;              // [nf] H rows (magnetic receivers)
  // forward injection (per source, merged duplicates)
  std::vector<Target> src_tg;
  std::vector<double> src_coef;          // one coefficient per target
  double src_scale = 1.0;
  // receiver nodes (shared by all sources)
  std::vector<int> rn_c;                 // component 0..2 (E) or 3..5 (H)
  std::vector<int64_t> rn_idx;
  std::vector<int> ri_ptr, ri_node;      // CSR over (r, ci) -> nodes
  std::vector<double> ri_w;
  // adjoint targets = receiver nodes; CSR node -> (row r*ncomp+ci, w / dual volume)
  std::vector<int> at_ptr, at_row;
  std::vector<double> at_w;

  // ---- basis functions ----
  bool have_basis = false;
  std::vector<double> basis;             // [2nf][nt]
  double gamma = 0, fit = 0;
  int basis_iters = 0;

  // ---- options ----
  int graph_steps = 32, bx = 64, by = 4, xcd = 1, strict_cfl = 1;   // bx: threads along x
  int kb = 8;                            // samples per volume-transform block (1, 2, 4, 8, 16, 32)
  int dec = 1, dec_log2 = 0;             // forward volume transform: every dec-th sample (2^dec_log2)
  int vx = 1;                            // E update: 1 x node per thread; 4: a 16-byte vector
  int vxh = 1;                           // the same for the H update
  int sched = 0;                         // 0: H and E launches per step; 1: one fused launch
  int kz = 8;                            // planes per block of the fused schedule
  int order = 0;                         // tile numbering: 0 x fastest, 1 z fastest
  int vti_grad = 0;                      // 1: gradients as [d/d ln rho_h, d/d ln rho_v]
  int lean = 1;                          // interior tiles take the lean update paths
  double barrier_us = 5.0e6;             // persistent schedule: longest wait at a grid barrier
  int persist_blocks = 0;                // persistent schedule: blocks per CU (0: occupancy)
  int barrier_sleep = 1;                 // persistent schedule: s_sleep units between polls
  int stream_stores = -1;                // non-temporal stores: 1 on, 0 off, -1 by working set
  bool streaming(bool with_vol) const;   // stream_stores resolved for a run
  int fd_order = 2;                      // order of the staggered differences: 2 or 4

  // ---- device side (managed in device.hip) ----
  void *dev = nullptr;
  uint64_t model_version = 0, basis_version = 0;
  double last_ms = 0;
  int last_steps = 0;
  int host_step = 0;          // steps completed in the current run (the device counters' value + 1)

  int64_t plane() const { return (int64_t)NY * PX; }
  int64_t field_elems() const { return (int64_t)NZ * NY * PX; }
  int64_t lin(int k, int j, int i) const { return ((int64_t)k * NY + j) * PX + i; }
  int nf() const { return (int)freqs.size(); }
  size_t tsize() const { return dtype == FWD_F64 ? 8 : 4; }
  size_t acc_bytes() const { return acc == FWD_ACC_F32 ? 8 : 16; }
  int64_t psi_elems_per_source() const;
  // transform-block history: samples 1 .. kb-1 of a block (the closing one
  // is read from the fields)
  int64_t hist_elems_per_source() const { return kb > 1 ? (int64_t)(kb - 1) * 3 * field_elems() : 0; }
  size_t core_state_bytes() const;  // fields + psi (double-buffered) + receiver sums + counters
  size_t state_bytes() const;       // core state + transform-block history
  size_t td_scratch_bytes(int segment) const;   // time-domain adjoint scratch
  size_t workspace_bytes(int mode) const;
  size_t volume_bytes() const;
};

// host setup (setup.cpp)
Plan *plan_create(const fwd_plan_desc *d);
void set_model(Plan &p, const double *rho, const double *rho_v = nullptr);
void basis_build(Plan &p, double gamma_rel, double gamma_abs, int max_iter, double tol,
                 double *fit_err, int *iters);
void get_table(const Plan &p, int which, double *out, size_t n);
// time-domain adjoint: receiver-node sensitivity coefficients [ns][nn][nf]
// (complex, scaled by a power of two) and 1/(sigma_e dV_e) per updated edge
void td_coefficients(const Plan &p, const double *resid, std::vector<double> &C,
                     double &scale);
void td_edge_weights(const Plan &p, std::vector<double> &W);

// device driver (device.hip)
void dev_release(Plan &p);
void dev_forward(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                 double *E_rec, void *stream);
void dev_forward_static(Plan &p, void *vol, size_t vol_bytes, double *E_rec, void *stream);
void dev_run_begin(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                   void *stream);
void dev_run_steps(Plan &p, void *ws, void *vol, int nsteps, void *stream);
void dev_run_receivers(Plan &p, void *ws, double *E_rec, void *stream);
void dev_run_flush(Plan &p, void *ws, void *vol, void *stream);
void dev_checkpoint(Plan &p, const void *ws, const void *vol, void *snap, int save,
                    void *stream);
void dev_volume_export(Plan &p, const void *vol, double *out, void *stream);
void dev_adjoint(Plan &p, void *ws, size_t ws_bytes, const void *vol, const double *resid,
                 double *grad, int accumulate, double *E_adj, void *stream);
void dev_adjoint_td(Plan &p, void *ws, size_t ws_bytes, void *scratch, size_t scratch_bytes,
                    int segment, const double *resid, double *grad, int accumulate,
                    void *stream);
double dev_autotune(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes,
                    int mode, int steps, void *stream);
void dev_set_sampling(Plan &p, int every);
int dev_get_sampling(Plan &p);
void dev_kernel_stats(Plan &p, double *ms3, int *count);

}  // namespace fwdem

struct fwd_plan {
  fwdem::Plan *p;
};
