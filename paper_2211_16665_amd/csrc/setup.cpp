// Host setup of a plan: validation, grid geometry, sigma -> fictitious
// permittivity, CFL time step, step count, CPML profiles, source wavelet and
// its transform, twiddles, injection/receiver tables, and the basis
// functions of the adjoint-source estimate (CGNR).  Pure host C++: no HIP.
//
// Paper references: Section 2 (eq. freq, eq. mittet and the correspondence
// sigma = 2 omega0 eps, eq. fictitiouswave, eq. dtft, eq. dft, the CPML of
// Komatitsch & Martin); Section 3.2-3.3 (eq. adj2, eq. B, eq. mpinv,
// eq. basis, the CGNR remark).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <sstream>
#include <unordered_map>

#include "fwdem_internal.hpp"

namespace fwdem {

void fail(fwd_status code, const std::string &msg) { throw Error{code, msg}; }

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int64_t Plan::psi_elems_per_source() const {
  const int64_t W = 2 * (int64_t)npml;
  return 4 * ((int64_t)NZ * NY * W + (int64_t)NZ * W * PX + W * (int64_t)NY * PX);
}

size_t Plan::core_state_bytes() const {
  // fields and CPML memory are double-buffered: step n reads half n % 2 and
  // writes the other half
  size_t b = align256(2 * (size_t)ns * 6 * field_elems() * tsize());
  b += align256(2 * (size_t)ns * psi_elems_per_source() * tsize());
  b += align256((size_t)ns * rn_c.size() * nf() * 16);
  b += 256;  // two step counters and the flush marker
  return b;
}

size_t Plan::state_bytes() const {
  return core_state_bytes() + align256((size_t)ns * hist_elems_per_source() * tsize());
}

size_t Plan::td_scratch_bytes(int segment) const {
  const size_t F = (size_t)field_elems(), nseg = ((size_t)nt + segment - 1) / segment;
  size_t b = nseg * align256(core_state_bytes());                        // checkpoints
  b += align256((size_t)(segment + 1) * ns * 3 * F * tsize());           // E of a segment
  b += align256((size_t)ns * 6 * F * tsize());                           // adjoint fields
  b += align256((size_t)ns * psi_elems_per_source() * tsize());          // adjoint CPML
  b += align256((size_t)ns * 3 * F * 8);                                 // gradient products
  b += align256((size_t)ns * rn_c.size() * nf() * 16);                   // sensitivities
  b += align256(3 * F * 8);                                              // edge weights
  return b;
}

size_t Plan::workspace_bytes(int mode) const {
  size_t b = state_bytes();
  // adjoint: gradient accumulators per source and edge (FP64)
  if (mode == FWD_MODE_ADJOINT) b += align256((size_t)ns * 3 * field_elems() * 8);
  return b;
}

size_t Plan::volume_bytes() const {
  return (size_t)ns * nf() * 3 * field_elems() * acc_bytes();
}

// Streaming stores pay when the data a step streams cannot stay in the
// 256 MB Infinity Cache until its next use: both field halves, and with a
// volume transform the history slots and the accumulators.
bool Plan::streaming(bool with_vol) const {
  if (stream_stores >= 0) return stream_stores == 1;
  const size_t tsize = dtype == FWD_F64 ? 8 : 4;
  size_t bytes = (size_t)ns * 12 * field_elems() * tsize;
  if (with_vol) bytes += (size_t)ns * 3 * field_elems() * tsize * (kb - 1) + volume_bytes();
  return bytes > ((size_t)256 << 20);
}

// ---------------------------------------------------------------------------
// plan creation
// ---------------------------------------------------------------------------
static void check_axis(const double *v, int n, const char *name) {
  if (!v) fail(FWD_ERR_INVALID_ARG, std::string("node array ") + name + " is NULL");
  for (int i = 0; i <= n; ++i) {
    if (!std::isfinite(v[i])) fail(FWD_ERR_INVALID_ARG, std::string(name) + " not finite");
    if (i > 0 && !(v[i] > v[i - 1]))
      fail(FWD_ERR_INVALID_ARG, std::string(name) + " nodes must increase strictly");
  }
}

// Metric lengths of the differences along one axis.  Order 2: cell widths
// and dual widths.  Order 4 (reading of the paper's high-order engine on a
// stretched grid, Section 2): the staggered pair (9/8, -1/24) in the index
// coordinate, so the metric is the same pair applied to the coordinates --
// of the nodes for the half-node metric, of the cell centres for the node
// metric -- with coordinates continued oddly across the two walls.
static void axis_metrics(Axis &ax, int order) {
  const int n = ax.n;
  ax.m = ax.h;
  ax.md = ax.hd;
  if (order != 4) return;
  const double c1 = 9.0 / 8.0, c2 = -1.0 / 24.0;
  const double x0 = ax.nodes[0], xn = ax.nodes[n];
  auto X = [&](int q) {                  // node coordinate, q in -1 .. n+1
    if (q < 0) return 2.0 * x0 - ax.nodes[-q];
    if (q > n) return 2.0 * xn - ax.nodes[2 * n - q];
    return ax.nodes[q];
  };
  auto C = [&](int q) {                  // cell centre, q in -2 .. n+1
    auto c = [&](int r) { return 0.5 * (ax.nodes[r] + ax.nodes[r + 1]); };
    if (q < 0) return 2.0 * x0 - c(-1 - q);
    if (q > n - 1) return 2.0 * xn - c(2 * n - 1 - q);
    return c(q);
  };
  for (int r = 0; r < n; ++r) ax.m[r] = c1 * (X(r + 1) - X(r)) + c2 * (X(r + 2) - X(r - 1));
  for (int i = 1; i < n; ++i) ax.md[i] = c1 * (C(i) - C(i - 1)) + c2 * (C(i + 1) - C(i - 2));
}

static void make_axis(Axis &ax, const double *v, int n) {
  ax.n = n;
  ax.nodes.assign(v, v + n + 1);
  ax.h.resize(n);
  for (int i = 0; i < n; ++i) ax.h[i] = v[i + 1] - v[i];
  ax.hd.resize(n + 1);
  ax.hd[0] = 0.5 * ax.h[0];
  ax.hd[n] = 0.5 * ax.h[n - 1];
  for (int i = 1; i < n; ++i) ax.hd[i] = 0.5 * (ax.h[i - 1] + ax.h[i]);
  axis_metrics(ax, 2);
}

Plan *plan_create(const fwd_plan_desc *d) {
  if (!d) fail(FWD_ERR_INVALID_ARG, "desc is NULL");
  if (d->npml < 0) fail(FWD_ERR_INVALID_ARG, "npml must be >= 0");
  const int nmin = 2 * d->npml + 4;
  if (d->nx < nmin || d->ny < nmin || d->nz < nmin)
    fail(FWD_ERR_INVALID_ARG, "each axis needs at least 2*npml+4 cells");
  if ((int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1) > (int64_t)1 << 34)
    fail(FWD_ERR_INVALID_ARG, "grid too large");
  check_axis(d->x, d->nx, "x");
  check_axis(d->y, d->ny, "y");
  check_axis(d->z, d->nz, "z");
  if (!(d->f0 > 0) || !std::isfinite(d->f0)) fail(FWD_ERR_INVALID_ARG, "f0 must be > 0");
  if (d->nfreq < 1 || d->nfreq > 64 || !d->freqs)
    fail(FWD_ERR_INVALID_ARG, "nfreq must be in [1, 64]");
  for (int k = 0; k < d->nfreq; ++k) {
    if (!(d->freqs[k] > 0) || !std::isfinite(d->freqs[k]))
      fail(FWD_ERR_INVALID_ARG, "frequencies must be > 0");
    for (int l = 0; l < k; ++l)
      if (d->freqs[l] == d->freqs[k]) fail(FWD_ERR_INVALID_ARG, "duplicate frequency");
  }
  if (d->nsrc < 1 || !d->src_pos || !d->src_mom) fail(FWD_ERR_INVALID_ARG, "need >= 1 source");
  if (d->nrec < 1 || !d->rec_pos) fail(FWD_ERR_INVALID_ARG, "need >= 1 receiver");
  if (d->ncomp < 1 || d->ncomp > 6 || !d->rec_comp) fail(FWD_ERR_INVALID_ARG, "ncomp in [1,6]");
  for (int c = 0; c < d->ncomp; ++c) {
    if (d->rec_comp[c] < 0 || d->rec_comp[c] > 5) fail(FWD_ERR_INVALID_ARG, "rec_comp in {0,...,5}");
    for (int e = 0; e < c; ++e)
      if (d->rec_comp[e] == d->rec_comp[c]) fail(FWD_ERR_INVALID_ARG, "duplicate receiver component");
  }
  if (d->field_dtype != FWD_F32 && d->field_dtype != FWD_F64)
    fail(FWD_ERR_INVALID_ARG, "field_dtype");
  if (d->acc_mode < FWD_ACC_F64 || d->acc_mode > FWD_ACC_F32) fail(FWD_ERR_INVALID_ARG, "acc_mode");
  if (d->dt < 0 || d->nt < 0) fail(FWD_ERR_INVALID_ARG, "dt and nt must be >= 0");
  if (d->src_kind != 0 && d->src_kind != 1) fail(FWD_ERR_INVALID_ARG, "src_kind in {0, 1}");

  Plan *p = new Plan();
  p->nx = d->nx;
  p->ny = d->ny;
  p->nz = d->nz;
  p->npml = d->npml;
  p->NX = d->nx + 1;
  p->NY = d->ny + 1;
  p->NZ = d->nz + 1;
  p->PX = (p->NX + 63) / 64 * 64;
  make_axis(p->ax[0], d->x, d->nx);
  make_axis(p->ax[1], d->y, d->ny);
  make_axis(p->ax[2], d->z, d->nz);
  p->cpml_order = d->cpml_order > 0 ? d->cpml_order : kCpmlOrder;
  p->cpml_R = d->cpml_R > 0 ? d->cpml_R : kCpmlR;
  p->cpml_kmax = d->cpml_kappa_max > 0 ? d->cpml_kappa_max : kCpmlKappaMax;
  p->cpml_amax_in = d->cpml_alpha_max;
  p->cpml_vref_in = d->cpml_vref;
  if (p->cpml_R >= 1.0) { delete p; fail(FWD_ERR_INVALID_ARG, "cpml_R must be < 1"); }
  p->f0 = d->f0;
  p->omega0 = 2.0 * kPi * d->f0;
  p->freqs.assign(d->freqs, d->freqs + d->nfreq);
  for (double f : p->freqs) {
    double w = 2.0 * kPi * f;
    p->omega.push_back(w);
    double a = std::sqrt(w * p->omega0);
    p->a.push_back(a);
    p->wprime.push_back(cplx(a, a));   // (1+i) sqrt(omega omega0)
  }
  p->ns = d->nsrc;
  p->nr = d->nrec;
  p->ncomp = d->ncomp;
  p->src_pos.assign(d->src_pos, d->src_pos + 3 * d->nsrc);
  p->src_mom.assign(d->src_mom, d->src_mom + 3 * d->nsrc);
  p->rec_pos.assign(d->rec_pos, d->rec_pos + 3 * d->nrec);
  p->comp.assign(d->rec_comp, d->rec_comp + d->ncomp);
  for (double v : p->src_pos) if (!std::isfinite(v)) { delete p; fail(FWD_ERR_INVALID_ARG, "src_pos"); }
  for (double v : p->src_mom) if (!std::isfinite(v)) { delete p; fail(FWD_ERR_INVALID_ARG, "src_mom"); }
  for (double v : p->rec_pos) if (!std::isfinite(v)) { delete p; fail(FWD_ERR_INVALID_ARG, "rec_pos"); }
  p->dtype = d->field_dtype;
  p->acc = d->acc_mode;
  p->cap = d->rho_air_cap > 0 ? d->rho_air_cap : kDefaultCap;
  p->cfl = d->cfl > 0 ? d->cfl : kDefaultCfl;
  if (p->cfl > 1.0) { delete p; fail(FWD_ERR_INVALID_ARG, "cfl must be <= 1"); }
  p->dt_user = d->dt;
  p->nt_user = d->nt;
  p->src_kind = d->src_kind;
  return p;
}

// ---------------------------------------------------------------------------
// model-dependent setup
// ---------------------------------------------------------------------------
// CPML coefficients at positions pos (Komatitsch & Martin, cited in Section 2):
// d = d0 r^m, d0 = -(m+1) vref ln R / (2L); kappa = 1 + (kmax-1) r^m;
// alpha = amax (1-r); b = exp(-(d/kappa + alpha) dt);
// a = d (b-1) / (kappa (d + kappa alpha)).
static void cpml_coeffs(const Plan &p, const Axis &ax, const std::vector<double> &pos,
                        std::vector<double> &kinv, std::vector<double> &b, std::vector<double> &a) {
  const int n = ax.n;
  const double xl = ax.nodes[p.npml], xr = ax.nodes[n - p.npml];
  const double Ll = std::max(xl - ax.nodes[0], 1e-300), Lr = std::max(ax.nodes[n] - xr, 1e-300);
  const double m = p.cpml_order;
  kinv.assign(pos.size(), 1.0);
  b.assign(pos.size(), 0.0);
  a.assign(pos.size(), 0.0);
  for (size_t q = 0; q < pos.size(); ++q) {
    double r, L;
    if (pos[q] < xl) {
      r = (xl - pos[q]) / Ll;
      L = Ll;
    } else if (pos[q] > xr) {
      r = (pos[q] - xr) / Lr;
      L = Lr;
    } else {
      continue;
    }
    const double d0 = -(m + 1.0) * p.vref * std::log(p.cpml_R) / (2.0 * L);
    const double dd = d0 * std::pow(r, m);
    const double kap = 1.0 + (p.cpml_kmax - 1.0) * std::pow(r, m);
    const double alp = p.amax * (1.0 - r);
    const double bb = std::exp(-(dd / kap + alp) * p.dt);
    kinv[q] = 1.0 / kap;
    b[q] = bb;
    a[q] = dd > 0.0 ? dd * (bb - 1.0) / (kap * (dd + kap * alp)) : 0.0;
  }
}

static void cpml_axis(const Plan &p, Axis &ax) {
  std::vector<double> mid(ax.n);
  for (int i = 0; i < ax.n; ++i) mid[i] = 0.5 * (ax.nodes[i] + ax.nodes[i + 1]);
  cpml_coeffs(p, ax, ax.nodes, ax.kinv_n, ax.b_n, ax.a_n);
  cpml_coeffs(p, ax, mid, ax.kinv_h, ax.b_h, ax.a_h);
}

// Trilinear weights on a lattice (positions l, increasing): index i with
// l[i] <= q <= l[i+1] and weights (1-t, t).
static void lin1(const std::vector<double> &l, double q, int &i, double &t) {
  if (!(q >= l.front() && q <= l.back())) fail(FWD_ERR_INVALID_ARG, "point outside the grid");
  i = (int)(std::upper_bound(l.begin(), l.end(), q) - l.begin()) - 1;
  i = std::min(i, (int)l.size() - 2);
  t = (q - l[i]) / (l[i + 1] - l[i]);
}

struct NodeW {
  int k, j, i;
  double w;
};

// Lattice of component c: E_x at (x_{i+1/2}, y_j, z_k) etc. for c = 0..2;
// H_x at (x_i, y_{j+1/2}, z_{k+1/2}) etc. for c = 3..5 (half nodes on the
// axes an E component has nodes on, and the reverse)
static std::vector<NodeW> point_weights(const Plan &p, int c, const double *q) {
  std::vector<double> lat[3];
  for (int d = 0; d < 3; ++d) {
    const Axis &ax = p.ax[d];
    if (c < 3 ? d == c : d != c - 3) {
      lat[d].resize(ax.n);
      for (int i = 0; i < ax.n; ++i) lat[d][i] = 0.5 * (ax.nodes[i] + ax.nodes[i + 1]);
    } else {
      lat[d] = ax.nodes;
    }
  }
  int id[3];
  double t[3];
  for (int d = 0; d < 3; ++d) lin1(lat[d], q[d], id[d], t[d]);
  std::vector<NodeW> out;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e) {
        double w = (a ? t[0] : 1 - t[0]) * (b ? t[1] : 1 - t[1]) * (e ? t[2] : 1 - t[2]);
        if (w != 0.0) out.push_back({id[2] + e, id[1] + b, id[0] + a, w});
      }
  return out;
}

// Is (k, j, i) an updated (non-boundary) edge of component c?
static bool interior_edge(const Plan &p, int c, int k, int j, int i) {
  switch (c) {
    case 0: return i >= 0 && i < p.nx && j >= 1 && j < p.ny && k >= 1 && k < p.nz;
    case 1: return i >= 1 && i < p.nx && j >= 0 && j < p.ny && k >= 1 && k < p.nz;
    default: return i >= 1 && i < p.nx && j >= 1 && j < p.ny && k >= 0 && k < p.nz;
  }
}

static double dual_volume(const Plan &p, int c, int k, int j, int i) {
  const Axis &X = p.ax[0], &Y = p.ax[1], &Z = p.ax[2];
  // in the metric lengths: the weights under which the discrete curl pair is
  // adjoint (cell and dual widths for order 2); an H node (c = 3..5) has the
  // node length on its own axis and cell lengths on the other two
  switch (c) {
    case 0: return X.m[i] * Y.md[j] * Z.md[k];
    case 1: return X.md[i] * Y.m[j] * Z.md[k];
    case 2: return X.md[i] * Y.md[j] * Z.m[k];
    case 3: return X.md[i] * Y.m[j] * Z.m[k];
    case 4: return X.m[i] * Y.md[j] * Z.m[k];
    default: return X.m[i] * Y.m[j] * Z.md[k];
  }
}

void set_model(Plan &p, const double *rho, const double *rho_v) {
  if (!rho) fail(FWD_ERR_INVALID_ARG, "rho is NULL");
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int64_t nc = (int64_t)nx * ny * nz;
  for (int64_t q = 0; q < nc; ++q)
    if (!(rho[q] > 0) || !std::isfinite(rho[q])) fail(FWD_ERR_INVALID_ARG, "rho must be finite and > 0");
  if (rho_v)
    for (int64_t q = 0; q < nc; ++q)
      if (!(rho_v[q] > 0) || !std::isfinite(rho_v[q]))
        fail(FWD_ERR_INVALID_ARG, "rho_v must be finite and > 0");
  for (int a = 0; a < 3; ++a) axis_metrics(p.ax[a], p.fd_order);
  const Axis &X = p.ax[0], &Y = p.ax[1], &Z = p.ax[2];
  const double old_dt = p.dt;
  const int old_nt = p.nt;

  p.rho.assign(rho, rho + nc);
  p.sigma.resize(nc);
  p.capped.resize(nc);
  // VTI (Section 2): sigma_h = sigma_xx = sigma_yy from rho, sigma_v =
  // sigma_zz from rho_v (isotropic when rho_v is NULL)
  p.vti = rho_v != nullptr;
  p.sigma_v.resize(nc);
  p.capped_v.resize(nc);
  double bound = std::numeric_limits<double>::infinity(), vmax = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int64_t q = ((int64_t)k * ny + j) * nx + i;
        const double r = std::min(rho[q], p.cap);    // air as cells at the capped resistivity
        p.capped[q] = rho[q] > p.cap;
        p.sigma[q] = 1.0 / r;
        const double rv = rho_v ? rho_v[q] : rho[q];
        p.capped_v[q] = rv > p.cap;
        p.sigma_v[q] = 1.0 / std::min(rv, p.cap);
        // fictitious wave speed v = 1/sqrt(mu eps), eps = sigma / (2 omega0),
        // taken along the faster (more resistive) direction of the cell
        const double v = std::sqrt(2.0 * p.omega0 / (kMu0 * std::min(p.sigma[q], p.sigma_v[q])));
        vmax = std::max(vmax, v);
        // order 4: the largest symbol of the difference grows by 9/8 + 1/24
        const double inv = (p.fd_order == 4 ? 7.0 / 6.0 : 1.0) *
                           std::sqrt(1.0 / (X.h[i] * X.h[i]) + 1.0 / (Y.h[j] * Y.h[j]) +
                                     1.0 / (Z.h[k] * Z.h[k]));
        bound = std::min(bound, 1.0 / (v * inv));
      }
  p.vmax = vmax;
  p.dt_cfl = bound;
  if (p.dt_user > 0) {
    if (p.strict_cfl && p.dt_user > bound)
      fail(FWD_ERR_CFL, "fixed dt exceeds the CFL bound of the model");
    p.dt = p.dt_user;
  } else {
    p.dt = p.cfl * bound;
  }
  double amin = *std::min_element(p.a.begin(), p.a.end());
  double amaxf = *std::max_element(p.a.begin(), p.a.end());
  if (p.nt_user > 0) {
    p.nt = p.nt_user;
  } else {
    double nt = std::ceil(std::log(1.0 / kNtTol) / (amin * p.dt));
    if (nt > 2.0e8) fail(FWD_ERR_INVALID_ARG, "derived step count above 2e8");
    p.nt = (int)nt;
  }
  p.vref = p.cpml_vref_in > 0 ? p.cpml_vref_in : vmax;
  p.amax = p.cpml_amax_in > 0 ? p.cpml_amax_in : kCpmlAlphaFactor * amin;
  for (int d = 0; d < 3; ++d) cpml_axis(p, p.ax[d]);

  // edge conductivity: volume-weighted mean of the cells sharing the edge;
  // dt/eps with eps = sigma / (2 omega0) on the edges the leapfrog updates
  const int64_t F = p.field_elems();
  for (int c = 0; c < 3; ++c) {
    p.sig_e[c].assign(F, 0.0);
    p.ce[c].assign(F, 0.0);
  }
  auto cellsig = [&](int k, int j, int i) { return p.sigma[((int64_t)k * ny + j) * nx + i]; };
  auto cellsig_v = [&](int k, int j, int i) { return p.sigma_v[((int64_t)k * ny + j) * nx + i]; };
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        const int64_t q = p.lin(k, j, i);
        // E_x: cells (k', j', i) with k' in {k-1, k}, j' in {j-1, j}
        if (i < nx) {
          double num = 0, den = 0;
          for (int kk = k - 1; kk <= k; ++kk)
            for (int jj = j - 1; jj <= j; ++jj)
              if (kk >= 0 && kk < nz && jj >= 0 && jj < ny) {
                const double w = Z.h[kk] * Y.h[jj];
                num += w * cellsig(kk, jj, i);
                den += w;
              }
          p.sig_e[0][q] = num / den;
          if (interior_edge(p, 0, k, j, i)) p.ce[0][q] = p.dt * 2.0 * p.omega0 / p.sig_e[0][q];
        }
        if (j < ny) {
          double num = 0, den = 0;
          for (int kk = k - 1; kk <= k; ++kk)
            for (int ii = i - 1; ii <= i; ++ii)
              if (kk >= 0 && kk < nz && ii >= 0 && ii < nx) {
                const double w = Z.h[kk] * X.h[ii];
                num += w * cellsig(kk, j, ii);
                den += w;
              }
          p.sig_e[1][q] = num / den;
          if (interior_edge(p, 1, k, j, i)) p.ce[1][q] = p.dt * 2.0 * p.omega0 / p.sig_e[1][q];
        }
        if (k < nz) {
          double num = 0, den = 0;
          for (int jj = j - 1; jj <= j; ++jj)
            for (int ii = i - 1; ii <= i; ++ii)
              if (jj >= 0 && jj < ny && ii >= 0 && ii < nx) {
                const double w = Y.h[jj] * X.h[ii];
                num += w * cellsig_v(k, jj, ii);   // z edges: vertical conductivity
                den += w;
              }
          p.sig_e[2][q] = num / den;
          if (interior_edge(p, 2, k, j, i)) p.ce[2][q] = p.dt * 2.0 * p.omega0 / p.sig_e[2][q];
        }
      }

  // wavelet: derivative of a Gaussian sampled at (n+1/2) dt (the paper leaves
  // the forward source time function open; outputs are normalised by its
  // transform W_k, so they do not depend on it)
  const int nf = p.nf(), nt = p.nt;
  p.tau = std::max(0.25 / amaxf, 3.0 * p.dt);
  p.t0 = 5.0 * p.tau;
  p.wavelet.resize(nt);
  for (int n = 0; n < nt; ++n) {
    const double u = ((n + 0.5) * p.dt - p.t0) / p.tau;
    p.wavelet[n] = -u * std::exp(-0.5 * u * u);
  }
  p.What.assign(nf, 0.0);
  p.norm.resize(nf);
  p.Omega.resize(nf);
  p.zE.resize((size_t)nt * nf);
  p.zH.resize((size_t)nt * nf);
  p.norm_h.resize(nf);
  const cplx I(0.0, 1.0);
  for (int k = 0; k < nf; ++k) {
    // electric sources inject J'^{n+1/2} = p w_n at (n+1/2) dt; magnetic
    // ones M'^n = m w_n at n dt (beside the curl E of the H update): each is
    // normalised by the transform of what it injects, when it injects it
    const double shift = p.src_kind == 1 ? 0.0 : 0.5;
    cplx acc = 0;
    for (int n = 0; n < nt; ++n) acc += p.wavelet[n] * std::exp(I * p.wprime[k] * ((n + shift) * p.dt));
    p.What[k] = acc;
    const cplx fac = std::sqrt(cplx(0.0, -p.omega[k] / (2.0 * p.omega0)));
    if (p.src_kind == 1) {
      // M' = M and E' = E: E = u / W^M; H' = sqrt(-i omega / 2 omega0) H
      p.norm[k] = 1.0 / acc;
      p.norm_h[k] = 1.0 / (fac * acc);
    } else {
      // J' = sqrt(-i omega / 2 omega0) J (correspondence below eq. mittet);
      // the magnetic field of the same source carries no sqrt factor
      p.norm[k] = fac / acc;
      p.norm_h[k] = 1.0 / acc;
    }
    p.Omega[k] = (2.0 / p.dt) * std::sin(p.wprime[k] * p.dt * 0.5);
    for (int n = 0; n < nt; ++n) {
      p.zE[(size_t)n * nf + k] = std::exp(I * p.wprime[k] * ((n + 1.0) * p.dt));
      p.zH[(size_t)n * nf + k] = std::exp(I * p.wprime[k] * ((n + 0.5) * p.dt));
    }
  }

  // forward injection: J = p delta(x - x_s) spread with trilinear weights
  // over each component's lattice, divided by the dual volume of the edge;
  // magnetic sources M = m delta(x - x_s) likewise over the H lattices and
  // the volumes of the H nodes (targets c = 3..5; every H node is updated)
  p.src_tg.clear();
  p.src_coef.clear();
  double cmax = 0;
  for (int s = 0; s < p.ns; ++s) {
    for (int cm = 0; cm < 3; ++cm) {
      const double m = p.src_mom[3 * s + cm];
      if (m == 0.0) continue;
      const int c = cm + 3 * p.src_kind;
      for (const NodeW &nw : point_weights(p, c, &p.src_pos[3 * s])) {
        if (c < 3 && !interior_edge(p, c, nw.k, nw.j, nw.i))
          fail(FWD_ERR_INVALID_ARG, "source touches the outer boundary of the grid");
        const int64_t idx = p.lin(nw.k, nw.j, nw.i);
        const double coef = m * nw.w / dual_volume(p, c, nw.k, nw.j, nw.i);
        bool merged = false;
        for (size_t t = 0; t < p.src_tg.size(); ++t)
          if (p.src_tg[t].s == s && p.src_tg[t].c == c && p.src_tg[t].idx == idx) {
            p.src_coef[t] += coef;
            merged = true;
          }
        if (!merged) {
          p.src_tg.push_back({s, c, idx, (int)p.src_coef.size()});
          p.src_coef.push_back(coef);
        }
      }
    }
  }
  for (size_t t = 0; t < p.src_tg.size(); ++t) {
    const Target &tg = p.src_tg[t];
    cmax = std::max(cmax, std::fabs(p.src_coef[t]) * (tg.c < 3 ? p.ce[tg.c][tg.idx] : p.dt / kMu0));
  }
  double wmax = 0;
  for (double w : p.wavelet) wmax = std::max(wmax, std::fabs(w));
  if (p.src_tg.empty() || cmax == 0) fail(FWD_ERR_INVALID_ARG, "every source moment is zero");
  // scale the injected current so the largest per-step increment of E is
  // near 1 (keeps single-precision fields far from the denormal range); a
  // power of two, so scaling and unscaling are exact, and undone in every
  // output
  p.src_scale = std::exp2(std::round(std::log2(1.0 / (cmax * wmax))));   // a power of two: exact

  // receivers: unique lattice nodes and the interpolation CSR
  p.rn_c.clear();
  p.rn_idx.clear();
  p.ri_ptr.assign(1, 0);
  p.ri_node.clear();
  p.ri_w.clear();
  std::vector<std::vector<std::pair<int, double>>> contrib;   // node -> (row, w/V)
  std::unordered_map<int64_t, int> node_of;
  for (int r = 0; r < p.nr; ++r)
    for (int ci = 0; ci < p.ncomp; ++ci) {
      const int c = p.comp[ci];
      for (const NodeW &nw : point_weights(p, c, &p.rec_pos[3 * r])) {
        // every H node is updated; E nodes on the outer walls are not
        if (c < 3 && !interior_edge(p, c, nw.k, nw.j, nw.i))
          fail(FWD_ERR_INVALID_ARG, "receiver touches the outer boundary of the grid");
        const int64_t idx = p.lin(nw.k, nw.j, nw.i);
        const int64_t key = idx * 6 + c;
        auto it = node_of.find(key);
        int node = it == node_of.end() ? -1 : it->second;
        if (node < 0) {
          node = (int)p.rn_c.size();
          node_of[key] = node;
          p.rn_c.push_back(c);
          p.rn_idx.push_back(idx);
          contrib.emplace_back();
        }
        p.ri_node.push_back(node);
        p.ri_w.push_back(nw.w);
        contrib[node].push_back({r * p.ncomp + ci, nw.w / dual_volume(p, c, nw.k, nw.j, nw.i)});
      }
      p.ri_ptr.push_back((int)p.ri_node.size());
    }
  p.at_ptr.assign(1, 0);
  p.at_row.clear();
  p.at_w.clear();
  for (auto &lst : contrib) {
    for (auto &rw : lst) {
      p.at_row.push_back(rw.first);
      p.at_w.push_back(rw.second);
    }
    p.at_ptr.push_back((int)p.at_row.size());
  }

  if (p.dt != old_dt || p.nt != old_nt) {
    p.have_basis = false;
    p.basis.clear();
  }
  p.have_model = true;
  p.model_version++;
}

// ---------------------------------------------------------------------------
// basis functions (Section 3.3): CGNR on the damped normal equations
//   (B^T B + gamma I) x = B^T e_j,  j = 0 .. 2 nf - 1
// with B applied from its rows (the damped cosines and sines of eq. B
// sampled at the injection times (n+1/2) dt), never forming B^T B.
// ---------------------------------------------------------------------------
void basis_build(Plan &p, double gamma_rel, double gamma_abs, int max_iter, double tol,
                 double *fit_err, int *iters) {
  if (!p.have_model) fail(FWD_ERR_STATE, "basis needs a model (dt and nt)");
  if (max_iter < 1 || !(tol > 0)) fail(FWD_ERR_INVALID_ARG, "max_iter >= 1 and tol > 0");
  if (gamma_abs < 0 || gamma_rel < 0) fail(FWD_ERR_INVALID_ARG, "gamma must be >= 0");
  const int nf = p.nf(), nt = p.nt, m = 2 * nf;
  std::vector<double> B((size_t)m * nt);
  double fro = 0;
  for (int k = 0; k < nf; ++k)
    for (int n = 0; n < nt; ++n) {
      const double t = (n + 0.5) * p.dt, at = p.a[k] * t, e = std::exp(-at);
      const double c = e * std::cos(at), s = e * std::sin(at);
      B[(size_t)k * nt + n] = c;
      B[(size_t)(nf + k) * nt + n] = s;
      fro += c * c + s * s;
    }
  const double gamma = gamma_abs > 0 ? gamma_abs : gamma_rel * fro;
  if (!(gamma > 0)) fail(FWD_ERR_INVALID_ARG, "gamma must be > 0");
  auto applyB = [&](const std::vector<double> &x, std::vector<double> &y) {
    for (int r = 0; r < m; ++r) {
      const double *row = &B[(size_t)r * nt];
      double acc = 0;
      for (int n = 0; n < nt; ++n) acc += row[n] * x[n];
      y[r] = acc;
    }
  };
  auto applyBt = [&](const std::vector<double> &y, std::vector<double> &x) {
    std::fill(x.begin(), x.end(), 0.0);
    for (int r = 0; r < m; ++r) {
      const double *row = &B[(size_t)r * nt];
      const double v = y[r];
      for (int n = 0; n < nt; ++n) x[n] += row[n] * v;
    }
  };
  auto dot = [](const std::vector<double> &a, const std::vector<double> &b) {
    double s = 0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
  };
  std::vector<double> basis((size_t)m * nt);
  std::vector<double> x(nt), r(m), s(nt), pdir(nt), q(m);
  int worst = 0;
  for (int col = 0; col < m; ++col) {
    // CGLS / CGNR (the paper's Claerbout conjugate gradient) for
    // min ||B x - e_col||^2 + gamma ||x||^2
    std::fill(x.begin(), x.end(), 0.0);
    std::fill(r.begin(), r.end(), 0.0);
    r[col] = 1.0;                    // r = e_col - B x
    applyBt(r, s);                   // s = B^T r - gamma x
    pdir = s;
    double g_old = dot(s, s);
    const double g0 = g_old;
    int it = 0;
    while (it < max_iter && g_old > tol * tol * g0) {
      applyB(pdir, q);
      const double delta = dot(q, q) + gamma * dot(pdir, pdir);
      if (!(delta > 0)) break;
      const double alpha = g_old / delta;
      for (int n = 0; n < nt; ++n) x[n] += alpha * pdir[n];
      for (int k = 0; k < m; ++k) r[k] -= alpha * q[k];
      applyBt(r, s);
      for (int n = 0; n < nt; ++n) s[n] -= gamma * x[n];
      const double g_new = dot(s, s);
      const double beta = g_new / g_old;
      for (int n = 0; n < nt; ++n) pdir[n] = s[n] + beta * pdir[n];
      g_old = g_new;
      ++it;
    }
    worst = std::max(worst, it);
    std::copy(x.begin(), x.end(), basis.begin() + (size_t)col * nt);
  }
  // fit: max |B B+ - I|
  double fit = 0;
  std::vector<double> y(m);
  for (int col = 0; col < m; ++col) {
    std::vector<double> xc(basis.begin() + (size_t)col * nt, basis.begin() + (size_t)(col + 1) * nt);
    applyB(xc, y);
    for (int k = 0; k < m; ++k) fit = std::max(fit, std::fabs(y[k] - (k == col ? 1.0 : 0.0)));
  }
  for (double v : basis)
    if (!std::isfinite(v)) fail(FWD_ERR_BASIS, "basis iteration produced a non-finite value");
  if (fit > 1e-2 && worst >= max_iter)
    fail(FWD_ERR_BASIS, "basis iteration did not converge (fit above 1e-2)");
  p.basis.swap(basis);
  p.gamma = gamma;
  p.fit = fit;
  p.basis_iters = worst;
  p.have_basis = true;
  p.basis_version++;
  if (fit_err) *fit_err = fit;
  if (iters) *iters = worst;
}

void td_coefficients(const Plan &p, const double *resid, std::vector<double> &C,
                     double &scale) {
  // E_rec[s][r][c][k] = norm_k sum_nodes w sum_m E^m z_k^m, so the misfit's
  // sensitivity to E^m at a node is -Re sum_k C_k z_k^m with
  // C_k = sum over the (receiver, component) rows touching the node of
  // w conj(resid) norm_k; magnetic rows likewise with norm_h and the samples
  // H^{n+1/2} z_k^{n+1/2}
  const int nf = p.nf(), nn = (int)p.rn_c.size(), rows = p.nr * p.ncomp;
  C.assign((size_t)p.ns * nn * nf * 2, 0.0);
  for (int s = 0; s < p.ns; ++s)
    for (int row = 0; row < rows; ++row)
      for (int e = p.ri_ptr[row]; e < p.ri_ptr[row + 1]; ++e) {
        const int node = p.ri_node[e];
        const bool mag = p.comp[row % p.ncomp] >= 3;   // H rows: H = norm_h sum H^{n+1/2} z^{n+1/2}
        for (int k = 0; k < nf; ++k) {
          const double *rr = &resid[2 * (((size_t)s * rows + row) * nf + k)];
          const cplx v = p.ri_w[e] * std::conj(cplx(rr[0], rr[1])) * (mag ? p.norm_h[k] : p.norm[k]);
          double *c = &C[2 * (((size_t)s * nn + node) * nf + k)];
          c[0] += v.real();
          c[1] += v.imag();
        }
      }
  double big = 0;
  for (double v : C) big = std::max(big, std::fabs(v));
  scale = big > 0 ? std::exp2(std::round(std::log2(1.0 / big))) : 1.0;   // power of two: exact
  for (double &v : C) v *= scale;
}

void td_edge_weights(const Plan &p, std::vector<double> &W) {
  const int64_t F = p.field_elems();
  W.assign(3 * F, 0.0);
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k <= p.nz; ++k)
      for (int j = 0; j <= p.ny; ++j)
        for (int i = 0; i <= p.nx; ++i)
          if (interior_edge(p, c, k, j, i)) {
            const int64_t q = p.lin(k, j, i);
            W[c * F + q] = 1.0 / (p.sig_e[c][q] * dual_volume(p, c, k, j, i));
          }
}

void get_table(const Plan &p, int which, double *out, size_t n) {
  auto need = [&](size_t m) {
    if (n < m) fail(FWD_ERR_INVALID_ARG, "output table too small");
  };
  if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
  switch (which) {
    case FWD_TAB_WAVELET:
      need(p.wavelet.size());
      std::copy(p.wavelet.begin(), p.wavelet.end(), out);
      break;
    case FWD_TAB_NORM:
    case FWD_TAB_OMEGA: {
      const std::vector<cplx> &v = which == FWD_TAB_NORM ? p.norm : p.Omega;
      need(2 * v.size());
      for (size_t k = 0; k < v.size(); ++k) {
        out[2 * k] = v[k].real();
        out[2 * k + 1] = v[k].imag();
      }
      break;
    }
    case FWD_TAB_CPML_X:
    case FWD_TAB_CPML_Y:
    case FWD_TAB_CPML_Z: {
      const Axis &ax = p.ax[which - FWD_TAB_CPML_X];
      const size_t w = ax.n + 1;
      need(6 * w);
      std::fill(out, out + 6 * w, 0.0);
      for (int i = 0; i <= ax.n; ++i) {
        out[i] = 1.0 / ax.kinv_n[i];
        out[w + i] = ax.b_n[i];
        out[2 * w + i] = ax.a_n[i];
      }
      for (int i = 0; i < ax.n; ++i) {
        out[3 * w + i] = 1.0 / ax.kinv_h[i];
        out[4 * w + i] = ax.b_h[i];
        out[5 * w + i] = ax.a_h[i];
      }
      break;
    }
    case FWD_TAB_BASIS:
      if (!p.have_basis) fail(FWD_ERR_BASIS, "no basis built");
      need(p.basis.size());
      std::copy(p.basis.begin(), p.basis.end(), out);
      break;
    case FWD_TAB_EDGE_SIGMA: {
      const size_t cells = (size_t)p.NZ * p.NY * p.NX;
      need(3 * cells);
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < p.NZ; ++k)
          for (int j = 0; j < p.NY; ++j)
            for (int i = 0; i < p.NX; ++i)
              out[c * cells + ((size_t)k * p.NY + j) * p.NX + i] = p.sig_e[c][p.lin(k, j, i)];
      break;
    }
    case FWD_TAB_METRIC_X:
    case FWD_TAB_METRIC_Y:
    case FWD_TAB_METRIC_Z: {
      const Axis &ax = p.ax[which - FWD_TAB_METRIC_X];
      const size_t w = ax.n + 1;
      need(2 * w);
      std::fill(out, out + 2 * w, 0.0);
      std::copy(ax.m.begin(), ax.m.end(), out);
      std::copy(ax.md.begin(), ax.md.end(), out + w);
      break;
    }
    default:
      fail(FWD_ERR_INVALID_ARG, "unknown table");
  }
}

}  // namespace fwdem
