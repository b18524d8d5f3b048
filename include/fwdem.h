/*
 * fwdem.h -- C ABI of the MI355X library for fictitious-wave-domain CSEM
 * modelling and its adjoint gradient (Yang, "3D fictitious wave domain
 * CSEM inversion by adjoint source estimation", arXiv 2211.16665).
 *
 * What the library computes
 *   forward  The diffusive frequency-domain Maxwell system (Section 2,
 *            eq. freq) is solved by stepping its fictitious wave-domain
 *            counterpart (eq. fictitiouswave, sigma = 2 omega0 eps, eq.
 *            mittet) with a staggered-grid E/H leapfrog on a stretched
 *            tensor grid with CPML layers, and extracting every frequency
 *            in one pass by the damped on-the-fly transform (eq. dft).
 *   adjoint  The adjoint field (eq. adj1, adj2) is stepped with the same
 *            engine, driven by time series built from the regularised
 *            basis functions B+ (Section 3.3, eqs. B, mpinv, basis), and the
 *            gradient of the misfit (eq. phid) with respect to ln(rho) is
 *            assembled from forward and adjoint fields (eq. gradsigmaij and
 *            the ln rho chain rule of Section 3.5).
 *
 * Conventions
 *   * Every call returns fwd_status; FWD_OK is 0.  On error a message is
 *     available from fwd_last_error() (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   * Grid: nx, ny, nz cells; node coordinates x[nx+1], y[ny+1], z[nz+1]
 *     strictly increasing (metres, z positive down).  Cell arrays are
 *     [nz][ny][nx], x fastest.
 *   * Complex numbers are interleaved (re, im) doubles.
 *   * Pointers named *_host are host memory read during the call; pointers
 *     named *_dev are device memory on the current HIP device.  Device
 *     buffers passed in (workspace, volume, outputs) are owned by the
 *     caller and must stay alive until the work enqueued on `stream` ends.
 *     Workspace, volume, scratch and snapshot buffers start on a 256-byte
 *     boundary (as hipMalloc returns them); others are rejected with
 *     FWD_ERR_INVALID_ARG.  The plan owns only tables proportional to one
 *     copy of the model.
 *   * Work is enqueued on the caller's stream (a hipStream_t passed as
 *     void*, 0 for the null stream).  fwd_forward / fwd_adjoint wait for
 *     their own work before returning, so that a non-finite result can be
 *     reported as FWD_ERR_NONFINITE.
 *   * fwd_plan_create, fwd_set_model, fwd_get_info, fwd_get_table and
 *     fwd_basis_build are host-only and make no HIP call.
 */
#ifndef FWDEM_H
#define FWDEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fwd_plan fwd_plan;

typedef enum {
  FWD_OK = 0,
  FWD_ERR_INVALID_ARG = 1,  /* argument outside its documented range */
  FWD_ERR_OOM = 2,          /* host or device allocation failed */
  FWD_ERR_HIP = 3,          /* a HIP runtime call failed */
  FWD_ERR_NONFINITE = 4,    /* the run produced Inf/NaN (e.g. dt above the CFL bound) */
  FWD_ERR_CFL = 5,          /* fixed dt above the CFL bound (FWD_OPT_STRICT_CFL on) */
  FWD_ERR_BASIS = 6,        /* basis functions missing or the iteration failed */
  FWD_ERR_UNSUPPORTED = 7,  /* combination of options not implemented */
  FWD_ERR_STATE = 8         /* call order violated (e.g. forward before set_model) */
} fwd_status;

enum { FWD_F32 = 0, FWD_F64 = 1 };                    /* field precision */
enum { FWD_ACC_F64 = 0, FWD_ACC_KAHAN = 1, FWD_ACC_F32 = 2 };  /* volume transform accumulators */
enum { FWD_MODE_FORWARD = 0, FWD_MODE_ADJOINT = 1 };

/* Problem description, copied by fwd_plan_create (the pointers are not kept). */
typedef struct {
  int nx, ny, nz;                 /* cells per axis, each >= 2*npml + 4 */
  const double *x, *y, *z;        /* host node coordinates (m) */
  int npml;                       /* CPML cells inside each end of each axis (>= 0) */
  /* CPML of Komatitsch & Martin (cited in Section 2); <= 0 selects the default
     order 2, R 1e-6, kappa_max 1, alpha_max 0.5 sqrt(omega_min omega0), vref =
     largest fictitious velocity of the model. */
  double cpml_order, cpml_R, cpml_kappa_max, cpml_alpha_max, cpml_vref;
  double f0;                      /* reference frequency omega0 / 2 pi (Hz), > 0 */
  int nfreq; const double *freqs; /* modelled frequencies (Hz), > 0, distinct */
  int nsrc;                       /* sources advanced together in one batch */
  const double *src_pos;          /* host [nsrc][3] dipole positions (m) */
  const double *src_mom;          /* host [nsrc][3] dipole moments (A m) */
  int nrec; const double *rec_pos;/* host [nrec][3] receiver positions (m) */
  int ncomp; const int *rec_comp; /* recorded components, distinct: 0, 1, 2 = E_x, E_y, E_z;
                                     3, 4, 5 = H_x, H_y, H_z (magnetic data, eq. phid W2) */
  int field_dtype;                /* FWD_F32 or FWD_F64 */
  int acc_mode;                   /* FWD_ACC_* for the volume transform */
  double rho_air_cap;             /* resistivities above the cap are stepped at the cap (<= 0: 1e4) */
  double cfl;                     /* fraction of the CFL bound used for dt (<= 0: 0.95) */
  double dt;                      /* > 0 fixes dt (s) instead of deriving it from the model */
  int nt;                         /* > 0 fixes the number of steps */
  int src_kind;                   /* 0: electric dipoles, J = p delta(x - x_s), moments in A m;
                                     1: magnetic dipoles, M = m delta(x - x_s) in the Faraday row
                                     of eq. freq (M' = M, eq. mittet), moments in V m, injected
                                     into the H update.  Every output is the field of the unit
                                     source of that kind. */
} fwd_plan_desc;

typedef struct {
  double dt, dt_cfl;              /* time step used and the CFL bound of the model */
  int nt;                         /* steps per run */
  double vmax, vref;              /* largest fictitious velocity, CPML reference velocity */
  double tau, t0;                 /* wavelet width and delay (s) */
  double src_scale;               /* internal source scaling undone in every output */
  int nx, ny, nz, px;             /* grid and padded x pitch of device arrays */
  int n_rec_nodes, n_src_entries, n_adj_targets;
  int have_basis, basis_iters;
  double basis_gamma, basis_fit;  /* gamma used and max |B B+ - I| */
  size_t workspace_bytes_forward, workspace_bytes_adjoint, volume_bytes, state_bytes;
} fwd_info;

/* Tables readable by fwd_get_table (host copies; for tests and tools). */
enum {
  FWD_TAB_WAVELET = 0,   /* [nt] w((n+1/2) dt) */
  FWD_TAB_NORM = 1,      /* complex [nfreq]: factor of the E rows; electric sources
                            sqrt(-i w / 2 w0) / W_k with W_k = sum_n w_n z_k^{n+1/2}, magnetic
                            1 / W^M_k with W^M_k = sum_n w_n z_k^n (H rows: either divided by
                            sqrt(-i w / 2 w0)) */
  FWD_TAB_OMEGA = 2,     /* complex [nfreq]: Omega_k = (2/dt) sin(w'_k dt/2) */
  FWD_TAB_CPML_X = 3,    /* [6][nx+1]: kappa, b, a at integer nodes, then at half nodes (last unused) */
  FWD_TAB_CPML_Y = 4,
  FWD_TAB_CPML_Z = 5,
  FWD_TAB_BASIS = 6,     /* [2 nfreq][nt] basis functions b_k (rows) */
  FWD_TAB_EDGE_SIGMA = 7, /* [3][nz+1][ny+1][nx+1] edge conductivity (x, y, z edges; unused slots 0) */
  FWD_TAB_METRIC_X = 8,   /* [2][nx+1]: metric lengths of the differences at the half nodes (last
                             unused), then at the nodes; cell and dual widths for order 2 */
  FWD_TAB_METRIC_Y = 9,
  FWD_TAB_METRIC_Z = 10
};

/* Validate `desc` and create a plan.  Host only.  Errors: INVALID_ARG. */
fwd_status fwd_plan_create(const fwd_plan_desc *desc, fwd_plan **plan_out);

/* Free the plan and its device tables (device work using it must be done). */
void fwd_plan_destroy(fwd_plan *plan);

/* Set the cell resistivity rho_host [nz][ny][nx] (ohm m, > 0).  Derives dt
 * (CFL, unless fixed), nt (damping of the lowest frequency to 1e-11, unless
 * fixed), CPML profiles, wavelet, twiddles and edge coefficients
 * (Section 2).  A change of dt or nt drops the basis functions.  Host only;
 * device tables are refreshed by the next device call. */
fwd_status fwd_set_model(fwd_plan *plan, const double *rho_host);

/* VTI model (Section 2: sigma_h = sigma_xx = sigma_yy, sigma_v = sigma_zz):
 * rho_h_host and rho_v_host [nz][ny][nx] (ohm m, > 0).  x and y edges average
 * 1/rho_h, z edges 1/rho_v; the CFL bound of a cell uses its faster (more
 * resistive) direction.  Otherwise as fwd_set_model.  Gradients
 * (fwd_adjoint, fwd_adjoint_td) are d phi / d ln rho with rho_h and rho_v
 * scaled together, or, with FWD_OPT_VTI_GRADIENT = 1, the pair
 * [d phi / d ln rho_h, d phi / d ln rho_v] (Section 3.1 VTI gradient: x and
 * y edges for rho_h, z edges for rho_v) in grad_dev [2][nz][ny][nx].
 * Errors: INVALID_ARG (NULL, non-positive or non-finite values), CFL. */
fwd_status fwd_set_model_vti(fwd_plan *plan, const double *rho_h_host,
                             const double *rho_v_host);

fwd_status fwd_get_info(const fwd_plan *plan, fwd_info *info);

/* Copy table `which` (FWD_TAB_*) into out_host (capacity n doubles). */
fwd_status fwd_get_table(const fwd_plan *plan, int which, double *out_host, size_t n);

/* Device bytes the caller provides as workspace for `mode` (FWD_MODE_*). */
fwd_status fwd_workspace_size(const fwd_plan *plan, int mode, size_t *bytes);

/* Device bytes of the forward volume transform (all sources, frequencies and
 * E components), the forward "wavefield checkpoint" the gradient needs. */
fwd_status fwd_volume_size(const fwd_plan *plan, size_t *bytes);

/* Full forward run: zero state, nt leapfrog steps, receiver output.
 *   ws_dev      workspace of fwd_workspace_size(FORWARD) bytes
 *   vol_dev     NULL, or fwd_volume_size bytes: receives the raw volume
 *               transform (layout private; read it with fwd_volume_export)
 *   E_rec_dev   complex [nsrc][nrec][ncomp][nfreq]: E(omega_k) of J = p delta
 *               (eq. freq) at the receivers, trilinear interpolation; rows
 *               of a magnetic component hold H(omega_k): the transform of
 *               H^{n+1/2} with z^{n+1/2} (eq. dtft lists H'), scaled by
 *               1 / W_k, since H' = sqrt(-i w/2w0) H (correspondence below
 *               eq. mittet) cancels the factor the E rows carry
 * Errors: STATE (no model), INVALID_ARG (sizes), HIP, NONFINITE. */
fwd_status fwd_forward(fwd_plan *plan, void *ws_dev, size_t ws_bytes,
                       void *vol_dev, size_t vol_bytes, double *E_rec_dev,
                       void *stream);

/* fwd_forward for callers that cannot allocate device memory (code under
 * HIP stream or graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same run, with the workspace in a static array of the
 * library's device code, FWD_STATIC_SCRATCH_BYTES per device, held by each
 * device the library runs on until the process ends.  It calls no hipMalloc,
 * hipFree or allocating routine: steps are launched one by one (no HIP
 * graph) and no timing is recorded (fwd_last_timing and fwd_kernel_stats
 * keep the values of the last fwd_forward / fwd_adjoint).
 *   vol_dev, vol_bytes, E_rec_dev, stream  as for fwd_forward (caller-owned)
 * Every call on one device uses that device's array, which keeps the last
 * call's contents (each call clears what it uses first): calls that overlap
 * on one device race.  The plan's device tables and entry lists must already
 * be on the current device for its current model and tiling options -- run
 * fwd_forward (or fwd_run_begin and fwd_run_steps) once after fwd_set_model
 * and after changing a tiling option; otherwise FWD_ERR_STATE.
 * Errors: STATE (no model, tables not resident), INVALID_ARG (the forward
 * workspace, fwd_workspace_size(FORWARD), needs more than
 * FWD_STATIC_SCRATCH_BYTES - 256 bytes; volume buffer too small), HIP,
 * NONFINITE. */
#define FWD_STATIC_SCRATCH_BYTES (32u << 20)
fwd_status fwd_forward_static(fwd_plan *plan, void *vol_dev, size_t vol_bytes, double *E_rec_dev,
                              void *stream);

/* Partial runs for checkpointing.  fwd_run_begin zeroes the state in ws;
 * vol is not cleared: the run's first transform block writes all of it (a
 * run flushed before its first sample clears it at the flush), so its
 * contents are defined once a block has closed or fwd_run_flush has
 * returned.  fwd_run_steps advances the state by nsteps (the step index
 * lives in the workspace, so runs may be split anywhere); fwd_run_receivers
 * writes the receiver output of the steps done so far, normalised as in
 * fwd_forward.  Only FWD_MODE_FORWARD runs can be split.  Every call takes
 * the byte counts of its buffers: a workspace below
 * fwd_workspace_size(FORWARD) or a volume buffer below fwd_volume_size is
 * refused with FWD_ERR_INVALID_ARG before any device work. */
fwd_status fwd_run_begin(fwd_plan *plan, void *ws_dev, size_t ws_bytes,
                         void *vol_dev, size_t vol_bytes, void *stream);
fwd_status fwd_run_steps(fwd_plan *plan, void *ws_dev, size_t ws_bytes, void *vol_dev,
                         size_t vol_bytes, int nsteps, void *stream);
fwd_status fwd_run_receivers(fwd_plan *plan, void *ws_dev, size_t ws_bytes, double *E_rec_dev,
                             void *stream);

/* Add the samples of an incomplete transform block (nsteps not a multiple of
 * FWD_OPT_DFT_BLOCK) to the volume transform, so that vol_dev holds the sum
 * over every step run so far (all zeros when the run has taken no sample
 * yet).  Stepping may continue afterwards: samples already added are not
 * added again.  fwd_forward does this itself. */
fwd_status fwd_run_flush(fwd_plan *plan, void *ws_dev, size_t ws_bytes, void *vol_dev,
                         size_t vol_bytes, void *stream);

/* Snapshot of the forward state (both halves of the double-buffered fields
 * and CPML memory, receiver sums, step index, transform-block history; the
 * volume transform when vol_dev is given): fwd_checkpoint_size bytes of
 * caller memory (device) per snapshot.  Buffers below their sizes (ws_bytes,
 * vol_bytes, snap_bytes) are refused with FWD_ERR_INVALID_ARG. */
fwd_status fwd_checkpoint_size(const fwd_plan *plan, int with_volume, size_t *bytes);
fwd_status fwd_checkpoint_save(fwd_plan *plan, const void *ws_dev, size_t ws_bytes,
                               const void *vol_dev, size_t vol_bytes, void *snap_dev,
                               size_t snap_bytes, void *stream);
fwd_status fwd_checkpoint_restore(fwd_plan *plan, void *ws_dev, size_t ws_bytes, void *vol_dev,
                                  size_t vol_bytes, const void *snap_dev, size_t snap_bytes,
                                  void *stream);

/* Normalised volume field E(omega_k) from a forward volume transform
 * (vol_bytes >= fwd_volume_size): out_dev complex
 * [nsrc][nfreq][3][nz+1][ny+1][nx+1]; component c sits at its staggered
 * position (E_x at (x_{i+1/2}, y_j, z_k), ...), slots outside a component's
 * lattice are 0. */
fwd_status fwd_volume_export(fwd_plan *plan, const void *vol_dev, size_t vol_bytes,
                             double *out_dev, void *stream);

/* Basis functions of the adjoint-source estimate (Section 3.3): the 2 nfreq
 * columns of B+ = (B^T B + gamma I)^-1 B^T, each obtained by a conjugate
 * gradient iteration on the damped normal equations (CGNR, as in the paper)
 * with B applied matrix-free.  Rows of B are sampled at the injection times
 * (n+1/2) dt.  gamma = gamma_abs if > 0, else gamma_rel * ||B||_F^2.
 * Iterates until the normal-equation residual falls below tol (relative) or
 * max_iter.  Host only.  Outputs (may be NULL): max |B B+ - I|, iterations
 * of the slowest column.  Errors: STATE (no model), BASIS (no convergence
 * and fit_err above 1e-2). */
fwd_status fwd_basis_build(fwd_plan *plan, double gamma_rel, double gamma_abs,
                           int max_iter, double tol, double *fit_err, int *iters);

/* Adjoint run and gradient.
 *   ws_dev        fwd_workspace_size(FWD_MODE_ADJOINT) bytes (ws_bytes)
 *   vol_fwd_dev   forward volume transform of the same model and sources,
 *                 vol_bytes >= fwd_volume_size
 *   resid_dev     complex [nsrc][nrec][ncomp][nfreq] weighted residual
 *                 W^2 (d - E) (eq. phid); for a general loss L(E) pass
 *                 -dL/dE (real and imaginary partial derivatives as re, im)
 *   grad_dev      double [nz][ny][nx]: d phi / d ln rho (Section 3.5) of the
 *                 misfit phi = 1/2 ||W (d - E)||^2, summed over sources;
 *                 added to the current content if accumulate != 0
 *   E_adj_dev     NULL or complex [nsrc][nrec][ncomp][nfreq]: transform of
 *                 the adjoint field at the receivers (raw, for checks)
 * The adjoint source at receiver r, component c is the time series
 * sum_k Re s_k b_k + Im s_k b_{k+nfreq} (eq. basis) of the spectrum
 * s_k = sqrt(-i omega_k / 2 omega0) conj(resid) (eq. adj2, electric
 * residual in the J' slot).  A magnetic residual (components 3-5) is a
 * magnetic current in the M' slot (M' = M), added to H at n dt before the
 * H update: its spectrum is s_k = conj(resid) z_k^{1/2}, because the basis
 * functions reproduce spectra at the J' times (n+1/2) dt, and its node
 * weights are w / (dual volume of the H node).  The coefficients are formed
 * from resid_dev on the device (no host copy of the residual); the call's
 * one synchronisation is the final non-finite check.  Errors: STATE (no
 * model / no basis), HIP, NONFINITE. */
fwd_status fwd_adjoint(fwd_plan *plan, void *ws_dev, size_t ws_bytes,
                       const void *vol_fwd_dev, size_t vol_bytes, const double *resid_dev,
                       double *grad_dev, int accumulate, double *E_adj_dev,
                       void *stream);

/* Time-domain adjoint and gradient (Appendix, alternative adjoint
 * formulation, applied to the stepped system): the exact derivative of
 * phi = 1/2 ||W (d - E)||^2 with respect to ln rho, with no basis
 * functions.  A forward run stores the core state (fields, CPML memory,
 * counters) every `segment` steps; then, from the last segment to the first,
 * the segment is replayed from its checkpoint and the transposed leapfrog
 * steps (including the transposed CPML recursions) run backward, driven at
 * the receiver nodes by d phi / d E^m = -Re sum_k C_k z_k^m, C_k = sum
 * w conj(resid) norm_k.  The gradient product on every updated edge is
 * sum_n Eadj^{n+1} (E^{n+1} - E^n) / sigma_e (discrete eq. chainrule),
 * mapped to cells by the transpose of the conductivity averaging.  Unlike
 * fwd_adjoint (eq. gradsigmaij) it is exact inside the CPML layers too.
 *   ws_dev       forward workspace, fwd_workspace_size(FWD_MODE_FORWARD)
 *   scratch_dev  fwd_adjoint_td_size(segment) bytes of device memory
 *                (checkpoints, the E of one segment, adjoint state)
 *   segment      steps between checkpoints (>= 1)
 *   resid_dev    complex [nsrc][nrec][ncomp][nfreq], W^2 (d - E)
 *   grad_dev     double [nz][ny][nx], added to if accumulate != 0
 * Magnetic receiver components add d phi / d H^{n+1/2} = -Re sum_k C_k
 * z_k^{n+1/2} (C_k with 1 / W_k) to the H multipliers of reverse step n.
 * Errors: STATE (no model), INVALID_ARG (sizes, segment), HIP.  Costs about
 * three forward runs (forward, replay, reverse sweep). */
fwd_status fwd_adjoint_td_size(const fwd_plan *plan, int segment, size_t *bytes);
fwd_status fwd_adjoint_td(fwd_plan *plan, void *ws_dev, size_t ws_bytes, void *scratch_dev,
                          size_t scratch_bytes, int segment, const double *resid_dev,
                          double *grad_dev, int accumulate, void *stream);

/* Tuning knobs (FWD_OPT_*); value semantics per key.  Host only. */
enum {
  FWD_OPT_GRAPH_STEPS = 0,   /* steps per captured HIP graph (0 or 1: launch eagerly); default 32 */
  FWD_OPT_BLOCK_X = 1,       /* threads per block along x: 16, 32, 64, 128 or 256.  x * y must
                                not exceed 256 when a run starts (else FWD_ERR_INVALID_ARG) */
  FWD_OPT_BLOCK_Y = 2,       /* block rows along y: 1, 2, 4, 8 or 16 */
  FWD_OPT_XCD_REMAP = 3,     /* 1: group neighbouring tiles on one XCD (default) */
  FWD_OPT_SAMPLE_EVERY = 4,  /* > 0: time the kernels of one step in every this many with
                                HIP events (those chunks launch eagerly); see fwd_kernel_stats */
  FWD_OPT_STRICT_CFL = 5,    /* 1 (default): fwd_set_model rejects a fixed dt above the CFL
                                bound with FWD_ERR_CFL; 0 lets it run (and typically end in
                                FWD_ERR_NONFINITE) */
  FWD_OPT_DFT_BLOCK = 6,     /* 1, 2, 4, 8 (default), 16 or 32: samples per read-modify-write of the
                                volume transform (and of the gradient product).  The E update
                                keeps samples 1 .. K-1 of a block in a history buffer of the
                                workspace; after the step whose sample closes the block, a
                                block-transform launch sums the K samples (FP64) and adds them
                                to the accumulators.  Changes only the order of the sums.  Set
                                it before fwd_workspace_size. */
  FWD_OPT_VECTOR = 7,        /* 1 (default): each thread of the E update updates one x node;
                                4: a 16-byte vector of consecutive x nodes (4 in FP32, 2 in
                                FP64); two-kernel schedule only */
  FWD_OPT_SCHEDULE = 8,      /* 0 (default): two launches per step (H update, then E update);
                                1: one fused launch per step -- each block owns a block_x x
                                block_y column tile and a chunk of FWD_OPT_ZCHUNK planes, stages
                                E and H planes with their halo in LDS and marches up in z,
                                recomputing the H halo of its tile;
                                2: persistent -- one cooperative launch runs up to 4096 steps,
                                every block looping over the tiles of schedule 0 (one node per
                                thread) through the H update, the E update and the block
                                transform, with a grid-wide barrier between phases (order 2,
                                transform block 8 or 16, vector widths forced to 1).
                                Same arithmetic per edge: results equal those of schedule 0 bit
                                for bit */
  FWD_OPT_ZCHUNK = 9,        /* planes per block of the fused schedule: 1 .. 64 (default 8) */
  FWD_OPT_TILE_ORDER = 10,   /* 0 (default): tiles numbered x fastest; 1: z fastest, so the
                                blocks of neighbouring planes run side by side */
  FWD_OPT_VECTOR_H = 11,     /* as FWD_OPT_VECTOR, for the H update */
  FWD_OPT_VTI_GRADIENT = 12, /* 0 (default): gradients [nz][ny][nx], d / d ln rho; 1: [2][nz][ny][nx],
                                d / d ln rho_h then d / d ln rho_v (see fwd_set_model_vti) */
  FWD_OPT_FD_ORDER = 13,     /* order of the staggered differences, 2 (default) or 4 (Section 2:
                                the paper's engine is high order on the stretched grid).  Order
                                4 uses the pair (9/8, -1/24) over the four nearest samples,
                                divided by metric lengths from the same pair on the
                                coordinates, with tangential E odd and H even across the walls;
                                the time step bound shrinks by 6/7.  Changing it drops the model
                                and the basis (call fwd_set_model again); order 4 runs the
                                two-kernel schedule with vector widths 1 and rejects other
                                SCHEDULE / VECTOR / VECTOR_H values. */
  FWD_OPT_LEAN = 14,         /* 1 (default): blocks of the two-kernel schedule whose tile lies
                                inside the CPML layers' inner boundary take an update path with
                                no CPML or wall logic; 0: every block takes the general path.
                                The arithmetic per edge is the same: results are equal bit for
                                bit. */
  FWD_OPT_BARRIER_US = 15,   /* persistent schedule: longest wait of a block at one grid barrier,
                                microseconds (default 5e6).  A longer wait (or a block that
                                gave up) ends the launch: every block returns and the call
                                reports FWD_ERR_HIP.  The run's state is then undefined. */
  FWD_OPT_PERSIST_BLOCKS = 16, /* persistent schedule: blocks per compute unit, 1 .. 32, or 0
                                (default) for as many as the occupancy of the kernel allows */
  FWD_OPT_BARRIER_SLEEP = 17, /* persistent schedule: pause between two polls of a waiting block,
                                in units of 64 clock cycles, 1 (default) .. 64 */
  FWD_OPT_DFT_DECIMATE = 18, /* D = 1 (default), 2, 4, ..., 64: forward runs add to the volume
                                transform only the samples E^m with m a multiple of D, each
                                weighted by D -- a coarser Riemann sum of eq. dtft than eq.
                                dft, an approximation that is not the paper's.  Its error is
                                the aliasing of the field's content above pi / (D dt): small
                                while D dt is well inside the source wavelet's width
                                (fwd_info.tau).  Receiver transforms and the adjoint's gradient
                                product take every sample (the adjoint sources of Section 3.3
                                start at full amplitude and would alias).  The E update keeps
                                history only on sampled steps and the block transform runs
                                once per D * FWD_OPT_DFT_BLOCK steps.  Schedule 0 only (other
                                schedules report FWD_ERR_UNSUPPORTED for forward runs with a
                                volume transform). */
  FWD_OPT_STREAM_STORES = 19 /* non-temporal (streaming) stores for the field halves and the
                                transform history in the H and E updates: 1 on, 0 off,
                                -1 (default) on when the bytes a step streams (both field
                                halves, and with a volume transform the history and the
                                accumulators) exceed the 256 MB Infinity Cache.  Results are
                                the same bit for bit either way.  On the 32 M-cell grid (8
                                sources) the hint speeds the H and E updates up by 5 % and 4 %;
                                on a grid whose data stay in the cache it slows them by 15-20 %:
                                a timed choice over a few steps proved unreliable, so the
                                autotuner leaves this option alone. */
};
fwd_status fwd_set_option(fwd_plan *plan, int key, double value);
fwd_status fwd_get_option(const fwd_plan *plan, int key, double *value);

/* Self-written tile/schedule autotuner.  A staged search on the given
 * buffers: block shape, then vector widths, then tile order and XCD remap,
 * then the fused schedule (shapes, planes per block), then the transform
 * block FWD_OPT_DFT_BLOCK in {8, 16, 32} when vol_dev is given and ws_bytes holds
 * the workspace of the longer block.  Each candidate runs `steps` steps of
 * the given mode untimed (graph capture) and then the same number timed; the
 * fastest is kept (as options of the plan) and its time per step (ms)
 * returned.  Results are cached for the life of the process, keyed by the
 * grid, sources, frequencies, precisions, order, mode and `steps`: a second
 * call with the same key only applies the cached choice.  The state in
 * ws/vol is clobbered.  The workspace size may change with the transform
 * block: query fwd_workspace_size again before the next run.  */
fwd_status fwd_autotune(fwd_plan *plan, void *ws_dev, size_t ws_bytes,
                        void *vol_dev, size_t vol_bytes, int mode, int steps,
                        double *best_ms, void *stream);

/* Kernel timing of the last fwd_forward / fwd_adjoint, measured with HIP
 * events on the caller's stream around the time-stepping region: total
 * milliseconds and number of steps. */
fwd_status fwd_last_timing(const fwd_plan *plan, double *ms, int *steps);

/* Average device time (ms) per launch of the kernels of a step over the
 * steps sampled in the last fwd_forward / fwd_adjoint (FWD_OPT_SAMPLE_EVERY >
 * 0): [0] H update, [1] E update (fused with injection and the receiver
 * transform; it keeps each sample for the volume transform), [2] block
 * transform (volume transform or gradient product of one transform block,
 * averaged over the sampled steps that closed a block; 0 if none).  Measured
 * with HIP events on the caller's stream that hipExtLaunchKernel stamps from
 * each sampled kernel's own dispatch (the kernel alone, as a kernel trace
 * reports it).  With the fused schedule [0] is 0 and [1] is the one launch
 * of the step.  avg_ms has room for 3 values. */
fwd_status fwd_kernel_stats(const fwd_plan *plan, double *avg_ms, int *samples);

const char *fwd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FWDEM_H */
