// Device side of the fictitious-wave-domain engine for gfx950 (MI355X).
//
// One leapfrog step (Section 2, eq. fictitiouswave) is four launches on the
// caller's stream:
//   k_update_h   H^{n+1/2} = H^{n-1/2} - dt/mu curl E^n            + CPML
//   k_inject     E^n -= dt/eps J'^{n+1/2} at the source (or adjoint-source)
//                edges, deterministic: one thread per target edge
//   k_update_e   E^{n+1} = E^n + dt/eps curl H^{n+1/2}               + CPML
//                fused with the volume transform acc_k += E^{n+1} z_k^{n+1}
//                (eq. dft) in the forward run, or with the on-the-fly gradient
//                product in the adjoint run
//   k_rec_dft    transform of E at the receiver lattice nodes
// The step index lives in device memory (incremented by k_update_h), so a
// captured HIP graph of K steps replays for any position in the run.
//
// The kernels are bound by HBM traffic (a 3D stencil plus an accumulator
// sweep, ~0.1-0.8 flop/byte): no matrix cores.  Threads own one (i, j, k)
// node of the padded layout [k][j][PX] (x fastest, PX a multiple of 64) and
// loop over the batched sources, so the per-edge coefficient is shared by
// all sources.  A 1D grid is remapped so that consecutive tiles of one XCD
// are spatial neighbours (their halos hit the same L2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fwdem_internal.hpp"

namespace fwdem {

#define HIP_CHECK(x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) fail(FWD_ERR_HIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// kernel parameter blocks
// ---------------------------------------------------------------------------
template <typename T>
struct AxisDev {
  const T *ih;     // 1/h   (n)
  const T *ihd;    // 1/hd  (n+1)
  const T *kn, *bn, *an;   // CPML at integer nodes: 1/kappa, b, a
  const T *kh, *bh, *ah;   // CPML at half nodes
};

template <typename T>
struct StepArgs {
  int nx, ny, nz, npml, PX, NY, NZ, ns;
  int64_t F;          // elements per field
  int64_t psi_src;    // psi elements per source
  T *fields;          // [ns][6][F]: Ex Ey Ez Hx Hy Hz
  T *psi;             // [ns][psi_src]
  const T *ce[3];     // dt/eps per edge component
  AxisDev<T> ax[3];
  T dtmu;             // dt / mu0
  const int *step;    // current step index (device)
  int *step_w;        // same, written by k_update_h
  // tiling
  int nbx, nby, nbz, nblocks, xcd;
  // volume transform / gradient
  int nf;
  const double2 *zE;  // [nt][nf] z^{n+1}
  void *vol;          // [ns][nf][3][F] accumulators (forward) or forward transform (adjoint)
  const double2 *Q;   // [nt][nf] gradient weights (adjoint)
  double *gedge;      // [3][F] gradient accumulators (adjoint)
  T *hist;            // [ns][kb-2][3][F] samples of the current transform block
  int64_t hist_src;   // history elements per source
  const int *flushed; // last sample already in the volume transform / gradient
};

__device__ __forceinline__ void tile_of(int nblocks, int xcd, int nbx, int nby, int &bx, int &by,
                                        int &bz) {
  int b = blockIdx.x;
  if (xcd) {
    // blocks are dealt round-robin to the 8 XCDs: give XCD x the tiles
    // [base_x, base_x + cnt_x) so its blocks are spatial neighbours
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, local = b >> 3;
    b = x * q + min(x, r) + local;
  }
  bx = b % nbx;
  const int t = b / nbx;
  by = t % nby;
  bz = t / nby;
}

// slab index of a CPML node: half nodes i+1/2 with i < npml or i >= n-npml;
// integer nodes with i < npml or i > n-npml; both map to [0, 2 npml)
__device__ __forceinline__ bool pml_half(int i, int n, int npml, int &l) {
  if (i < npml) { l = i; return true; }
  if (i >= n - npml) { l = i - n + 2 * npml; return true; }
  return false;
}
__device__ __forceinline__ bool pml_int(int i, int n, int npml, int &l) {
  if (i < npml) { l = i; return true; }
  if (i > n - npml) { l = i - n + 2 * npml - 1; return true; }
  return false;
}

// ---------------------------------------------------------------------------
// H update: H^{n+1/2} = H^{n-1/2} - dt/mu (curl E^n)
//   H_x -= dt/mu (dEz/dy - dEy/dz), H_y -= dt/mu (dEx/dz - dEz/dx),
//   H_z -= dt/mu (dEy/dx - dEx/dy); forward differences over a cell width
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_update_h(StepArgs<T> A) {
  int bx, by, bz;
  if ((int)blockIdx.x >= A.nblocks) return;
  tile_of(A.nblocks, A.xcd, A.nbx, A.nby, bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz;
  if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) A.step_w[0] = A.step_w[0] + 1;
  if (i > A.nx || j > A.ny || k > A.nz) return;
  const int PX = A.PX, NY = A.NY, NZ = A.NZ, npml = A.npml, W = 2 * npml;
  const int64_t plane = (int64_t)NY * PX;
  const int64_t q = (int64_t)k * plane + (int64_t)j * PX + i;
  const T dtmu = A.dtmu;
  const AxisDev<T> &X = A.ax[0], &Y = A.ax[1], &Z = A.ax[2];
  const bool hx_ok = j < A.ny && k < A.nz;
  const bool hy_ok = i < A.nx && k < A.nz;
  const bool hz_ok = i < A.nx && j < A.ny;
  int lx = 0, ly = 0, lz = 0;
  const bool px = npml > 0 && pml_half(i, A.nx, npml, lx);
  const bool py = npml > 0 && pml_half(j, A.ny, npml, ly);
  const bool pz = npml > 0 && pml_half(k, A.nz, npml, lz);
  const int64_t sX = (int64_t)NZ * NY * W, sY = (int64_t)NZ * W * PX, sZ = (int64_t)W * NY * PX;
  for (int s = 0; s < A.ns; ++s) {
    T *f = A.fields + (int64_t)s * 6 * A.F;
    const T *ex = f, *ey = f + A.F, *ez = f + 2 * A.F;
    T *hx = f + 3 * A.F, *hy = f + 4 * A.F, *hz = f + 5 * A.F;
    T *ps = A.psi + (int64_t)s * A.psi_src;
    T *psX = ps, *psY = ps + 4 * sX, *psZ = psY + 4 * sY;
    const int64_t iX = ((int64_t)k * NY + j) * W + lx;
    const int64_t iY = ((int64_t)k * W + ly) * PX + i;
    const int64_t iZ = ((int64_t)lz * NY + j) * PX + i;
    if (hx_ok) {
      T d1 = (ez[q + PX] - ez[q]) * Y.ih[j];     // dEz/dy at y_{j+1/2}
      T d2 = (ey[q + plane] - ey[q]) * Z.ih[k];  // dEy/dz at z_{k+1/2}
      if (py) { T &p = psY[0 * sY + iY]; p = Y.bh[j] * p + Y.ah[j] * d1; d1 = d1 * Y.kh[j] + p; }
      if (pz) { T &p = psZ[0 * sZ + iZ]; p = Z.bh[k] * p + Z.ah[k] * d2; d2 = d2 * Z.kh[k] + p; }
      hx[q] -= dtmu * (d1 - d2);
    }
    if (hy_ok) {
      T d1 = (ex[q + plane] - ex[q]) * Z.ih[k];  // dEx/dz
      T d2 = (ez[q + 1] - ez[q]) * X.ih[i];      // dEz/dx
      if (pz) { T &p = psZ[1 * sZ + iZ]; p = Z.bh[k] * p + Z.ah[k] * d1; d1 = d1 * Z.kh[k] + p; }
      if (px) { T &p = psX[0 * sX + iX]; p = X.bh[i] * p + X.ah[i] * d2; d2 = d2 * X.kh[i] + p; }
      hy[q] -= dtmu * (d1 - d2);
    }
    if (hz_ok) {
      T d1 = (ey[q + 1] - ey[q]) * X.ih[i];      // dEy/dx
      T d2 = (ex[q + PX] - ex[q]) * Y.ih[j];     // dEx/dy
      if (px) { T &p = psX[1 * sX + iX]; p = X.bh[i] * p + X.ah[i] * d1; d1 = d1 * X.kh[i] + p; }
      if (py) { T &p = psY[1 * sY + iY]; p = Y.bh[j] * p + Y.ah[j] * d2; d2 = d2 * Y.kh[j] + p; }
      hz[q] -= dtmu * (d1 - d2);
    }
  }
}

// ---------------------------------------------------------------------------
// accumulator flavours for the volume transform acc += E z (eq. dft)
// ---------------------------------------------------------------------------
enum { ACC_NONE = 0, ACC_F64 = 1, ACC_KAHAN = 2, ACC_F32 = 3 };

template <int ACC>
__device__ __forceinline__ void acc_add(void *base, int64_t idx, double2 x) {
  if constexpr (ACC == ACC_F64) {
    double2 *p = reinterpret_cast<double2 *>(base) + idx;
    double2 v = *p;
    v.x += x.x;
    v.y += x.y;
    *p = v;
  } else if constexpr (ACC == ACC_KAHAN) {
    // compensated single precision: (hi, lo) per real component, the sum is
    // hi - lo (Kahan's running compensation)
    float4 *p = reinterpret_cast<float4 *>(base) + idx;
    float4 v = *p;
    const float xr = (float)x.x, xi = (float)x.y;
    float yr = xr - v.z, tr = v.x + yr;
    v.z = (tr - v.x) - yr;
    v.x = tr;
    float yi = xi - v.w, ti = v.y + yi;
    v.w = (ti - v.y) - yi;
    v.y = ti;
    *p = v;
  } else if constexpr (ACC == ACC_F32) {
    float2 *p = reinterpret_cast<float2 *>(base) + idx;
    float2 v = *p;
    v.x += (float)x.x;
    v.y += (float)x.y;
    *p = v;
  }
}

template <int ACC>
__device__ __forceinline__ double2 acc_read(const void *base, int64_t idx) {
  if constexpr (ACC == ACC_F64) {
    return reinterpret_cast<const double2 *>(base)[idx];
  } else if constexpr (ACC == ACC_KAHAN) {
    const float4 v = reinterpret_cast<const float4 *>(base)[idx];
    return make_double2((double)v.x - (double)v.z, (double)v.y - (double)v.w);
  } else {
    const float2 v = reinterpret_cast<const float2 *>(base)[idx];
    return make_double2((double)v.x, (double)v.y);
  }
}

// After the E update of component c at q (old value e0 = sample m-1, new
// value e1 = sample m, m = n+1): the transform over a block of KB samples
// is added in one read-modify-write when the block closes (m % KB == 0);
// samples with m % KB in 1..KB-2 wait in the history buffer, the sample
// with m % KB == KB-1 is the old value of the closing step.  KB = 1 adds
// every sample as it comes.  Forward: volume transform acc_k += sum E z_k^m
// (eq. dft).  Adjoint: g += sum_m u^m Re(sum_k Q_k^m V_k), the gradient
// product of eq. gradsigmaij accumulated over time (Q on the host).
// Samples at or before *flushed were already added by a flush.
template <typename T, int ACC, bool ADJ, int KB>
__device__ __forceinline__ void post_e(const StepArgs<T> &A, int s, int c, int64_t q, T e0, T e1,
                                       int n, double &g) {
  if constexpr (ACC != ACC_NONE) {
    const int nf = A.nf;
    const int m = n + 1;
    const int r = m & (KB - 1);
    T *h = A.hist + (int64_t)s * A.hist_src + (int64_t)c * A.F + q;
    if constexpr (KB > 1) {
      if (r != 0) {
        if (r <= KB - 2) h[(int64_t)(r - 1) * 3 * A.F] = e1;
        return;
      }
    }
    // the KB samples of the block: m-KB+1 .. m; zE / Q index = sample - 1
    double val[KB];
#pragma unroll
    for (int t = 0; t < KB - 2; ++t) val[t] = (double)h[(int64_t)t * 3 * A.F];
    if constexpr (KB >= 2) val[KB - 2] = (double)e0;
    val[KB - 1] = (double)e1;
    const int fl = A.flushed[0];
    const int first = m - KB + 1;
#pragma unroll
    for (int t = 0; t < KB; ++t)
      if (first + t <= fl) val[t] = 0.0;
    const int64_t base = ((int64_t)s * nf * 3 + c) * A.F + q;
    if constexpr (!ADJ) {
      for (int kf = 0; kf < nf; ++kf) {
        double2 sum = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < KB; ++t) {
          const double2 z = A.zE[(int64_t)(first - 1 + t) * nf + kf];
          sum.x = fma(val[t], z.x, sum.x);
          sum.y = fma(val[t], z.y, sum.y);
        }
        acc_add<ACC>(A.vol, base + (int64_t)kf * 3 * A.F, sum);
      }
    } else {
      double re = 0.0;
      for (int kf = 0; kf < nf; ++kf) {
        const double2 v = acc_read<ACC>(A.vol, base + (int64_t)kf * 3 * A.F);
#pragma unroll
        for (int t = 0; t < KB; ++t) {
          const double2 Qt = A.Q[(int64_t)(first - 1 + t) * nf + kf];
          re = fma(val[t], Qt.x * v.x - Qt.y * v.y, re);
        }
      }
      g += re;
    }
  }
}

// ---------------------------------------------------------------------------
// E update: E^{n+1} = E^n + dt/eps curl H^{n+1/2} on interior edges
//   E_x += ce (dHz/dy - dHy/dz), E_y += ce (dHx/dz - dHz/dx),
//   E_z += ce (dHy/dx - dHx/dy); backward differences over a dual width
// ---------------------------------------------------------------------------
template <typename T, int ACC, bool ADJ, int KB>
__global__ void __launch_bounds__(256) k_update_e(StepArgs<T> A) {
  int bx, by, bz;
  if ((int)blockIdx.x >= A.nblocks) return;
  tile_of(A.nblocks, A.xcd, A.nbx, A.nby, bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz;
  if (i > A.nx || j > A.ny || k > A.nz) return;
  const int PX = A.PX, NY = A.NY, NZ = A.NZ, npml = A.npml, W = 2 * npml;
  const int64_t plane = (int64_t)NY * PX;
  const int64_t q = (int64_t)k * plane + (int64_t)j * PX + i;
  const int n = A.step[0];
  const AxisDev<T> &X = A.ax[0], &Y = A.ax[1], &Z = A.ax[2];
  const bool ex_ok = i < A.nx && j >= 1 && j < A.ny && k >= 1 && k < A.nz;
  const bool ey_ok = i >= 1 && i < A.nx && j < A.ny && k >= 1 && k < A.nz;
  const bool ez_ok = i >= 1 && i < A.nx && j >= 1 && j < A.ny && k < A.nz;
  int lx = 0, ly = 0, lz = 0;
  const bool px = npml > 0 && pml_int(i, A.nx, npml, lx);
  const bool py = npml > 0 && pml_int(j, A.ny, npml, ly);
  const bool pz = npml > 0 && pml_int(k, A.nz, npml, lz);
  const int64_t sX = (int64_t)NZ * NY * W, sY = (int64_t)NZ * W * PX, sZ = (int64_t)W * NY * PX;
  const T cex = ex_ok ? A.ce[0][q] : T(0), cey = ey_ok ? A.ce[1][q] : T(0),
          cez = ez_ok ? A.ce[2][q] : T(0);
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int s = 0; s < A.ns; ++s) {
    T *f = A.fields + (int64_t)s * 6 * A.F;
    T *ex = f, *ey = f + A.F, *ez = f + 2 * A.F;
    const T *hx = f + 3 * A.F, *hy = f + 4 * A.F, *hz = f + 5 * A.F;
    T *ps = A.psi + (int64_t)s * A.psi_src;
    T *psX = ps, *psY = ps + 4 * sX, *psZ = psY + 4 * sY;
    const int64_t iX = ((int64_t)k * NY + j) * W + lx;
    const int64_t iY = ((int64_t)k * W + ly) * PX + i;
    const int64_t iZ = ((int64_t)lz * NY + j) * PX + i;
    if (ex_ok) {
      T d1 = (hz[q] - hz[q - PX]) * Y.ihd[j];     // dHz/dy at y_j
      T d2 = (hy[q] - hy[q - plane]) * Z.ihd[k];  // dHy/dz at z_k
      if (py) { T &p = psY[2 * sY + iY]; p = Y.bn[j] * p + Y.an[j] * d1; d1 = d1 * Y.kn[j] + p; }
      if (pz) { T &p = psZ[2 * sZ + iZ]; p = Z.bn[k] * p + Z.an[k] * d2; d2 = d2 * Z.kn[k] + p; }
      const T e0 = ex[q];
      const T e = e0 + cex * (d1 - d2);
      ex[q] = e;
      post_e<T, ACC, ADJ, KB>(A, s, 0, q, e0, e, n, gx);
    }
    if (ey_ok) {
      T d1 = (hx[q] - hx[q - plane]) * Z.ihd[k];  // dHx/dz
      T d2 = (hz[q] - hz[q - 1]) * X.ihd[i];      // dHz/dx
      if (pz) { T &p = psZ[3 * sZ + iZ]; p = Z.bn[k] * p + Z.an[k] * d1; d1 = d1 * Z.kn[k] + p; }
      if (px) { T &p = psX[2 * sX + iX]; p = X.bn[i] * p + X.an[i] * d2; d2 = d2 * X.kn[i] + p; }
      const T e0 = ey[q];
      const T e = e0 + cey * (d1 - d2);
      ey[q] = e;
      post_e<T, ACC, ADJ, KB>(A, s, 1, q, e0, e, n, gy);
    }
    if (ez_ok) {
      T d1 = (hy[q] - hy[q - 1]) * X.ihd[i];      // dHy/dx
      T d2 = (hx[q] - hx[q - PX]) * Y.ihd[j];     // dHx/dy
      if (px) { T &p = psX[3 * sX + iX]; p = X.bn[i] * p + X.an[i] * d1; d1 = d1 * X.kn[i] + p; }
      if (py) { T &p = psY[3 * sY + iY]; p = Y.bn[j] * p + Y.an[j] * d2; d2 = d2 * Y.kn[j] + p; }
      const T e0 = ez[q];
      const T e = e0 + cez * (d1 - d2);
      ez[q] = e;
      post_e<T, ACC, ADJ, KB>(A, s, 2, q, e0, e, n, gz);
    }
  }
  if constexpr (ADJ) {
    if (((n + 1) & (KB - 1)) == 0) {
      if (ex_ok) A.gedge[q] += gx;
      if (ey_ok) A.gedge[A.F + q] += gy;
      if (ez_ok) A.gedge[2 * A.F + q] += gz;
    }
  }
}

// Flush: add the samples of the incomplete last block (m_last % KB != 0)
// that are newer than *flushed; the caller then moves *flushed to m_last
// with k_set_flushed.  Same thread mapping as the E update.
template <typename T, int ACC, bool ADJ, int KB>
__global__ void __launch_bounds__(256) k_flush(StepArgs<T> A) {
  int bx, by, bz;
  if ((int)blockIdx.x >= A.nblocks) return;
  tile_of(A.nblocks, A.xcd, A.nbx, A.nby, bx, by, bz);
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  const int k = bz;
  if (i > A.nx || j > A.ny || k > A.nz) return;
  const int m_last = A.step[0] + 1;
  const int r_end = m_last & (KB - 1);
  if (KB == 1 || r_end == 0) return;
  const int fl = A.flushed[0];
  const int64_t q = ((int64_t)k * A.NY + j) * A.PX + i;
  const bool ok[3] = {i < A.nx && j >= 1 && j < A.ny && k >= 1 && k < A.nz,
                      i >= 1 && i < A.nx && j < A.ny && k >= 1 && k < A.nz,
                      i >= 1 && i < A.nx && j >= 1 && j < A.ny && k < A.nz};
  const int nf = A.nf;
  double g[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < A.ns; ++s) {
    const T *f = A.fields + (int64_t)s * 6 * A.F;
    for (int c = 0; c < 3; ++c) {
      if (!ok[c]) continue;
      const T *h = A.hist + (int64_t)s * A.hist_src + (int64_t)c * A.F + q;
      const int64_t base = ((int64_t)s * nf * 3 + c) * A.F + q;
      for (int rr = 1; rr <= r_end; ++rr) {
        const int mm = m_last - r_end + rr;
        if (mm <= fl) continue;
        const double v = rr <= KB - 2 ? (double)h[(int64_t)(rr - 1) * 3 * A.F]
                                      : (double)f[(int64_t)c * A.F + q];
        for (int kf = 0; kf < nf; ++kf) {
          if constexpr (!ADJ) {
            const double2 z = A.zE[(int64_t)(mm - 1) * nf + kf];
            acc_add<ACC>(A.vol, base + (int64_t)kf * 3 * A.F, make_double2(v * z.x, v * z.y));
          } else {
            const double2 Vk = acc_read<ACC>(A.vol, base + (int64_t)kf * 3 * A.F);
            const double2 Qt = A.Q[(int64_t)(mm - 1) * nf + kf];
            g[c] += v * (Qt.x * Vk.x - Qt.y * Vk.y);
          }
        }
      }
    }
  }
  if constexpr (ADJ) {
    for (int c = 0; c < 3; ++c)
      if (ok[c]) A.gedge[(int64_t)c * A.F + q] += g[c];
  }
}

__global__ void k_set_flushed(int *flushed, const int *step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flushed[0] = step[0] + 1;
}

// ---------------------------------------------------------------------------
// injection of J'^{n+1/2}: E -= ce * sum_r coef[toff+r] F[r][n]
// Forward: one thread per (source, component, edge) target; adjoint: one
// thread per (component, edge) node looping over the sources.  No atomics.
// The E update that follows reads the injected value as its "old" sample
// E^n; when a transform block closes at this step (KB > 1) the exact
// difference E^n - (E^n - ce J) is added here to the volume transform
// (forward) or to the gradient product (adjoint) at the target edge.
// ---------------------------------------------------------------------------
template <typename T>
struct InjArgs {
  int ntg, nrow, nt, ns, nn, nf;
  const int *tg_s, *tg_c, *tg_toff;
  const int64_t *tg_idx;
  const double *coef, *Ftab;
  T *fields;
  int64_t F;
  const T *ce0, *ce1, *ce2;
  const int *step, *flushed;
  void *vol;
  const double2 *zE, *Q;
  double *gedge;
};

template <typename T, int ACC, bool ADJ, int KB>
__global__ void k_inject(InjArgs<T> I) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= I.ntg) return;
  const int n = I.step[0];
  const bool closing = ACC != ACC_NONE && KB > 1 && ((n + 1) & (KB - 1)) == 0 && n > I.flushed[0];
  const int c = I.tg_c[t];
  const int64_t idx = I.tg_idx[t];
  const T *ce = c == 0 ? I.ce0 : (c == 1 ? I.ce1 : I.ce2);
  const double cev = (double)ce[idx];
  const int nf = I.nf;
  if constexpr (!ADJ) {
    const int s = I.tg_s[t];
    double v = 0.0;
    const double *cf = I.coef + I.tg_toff[t];
    for (int r = 0; r < I.nrow; ++r) v += cf[r] * I.Ftab[(int64_t)r * I.nt + n];
    T *E = I.fields + ((int64_t)s * 6 + c) * I.F;
    const T old = E[idx];
    const T now = old - (T)(cev * v);
    E[idx] = now;
    if constexpr (ACC != ACC_NONE) {
      if (closing) {
        const double dlt = (double)old - (double)now;
        const int64_t base = (((int64_t)s * nf) * 3 + c) * I.F + idx;
        for (int kf = 0; kf < nf; ++kf) {
          const double2 z = I.zE[(int64_t)(n - 1) * nf + kf];
          acc_add<ACC>(I.vol, base + (int64_t)kf * 3 * I.F, make_double2(dlt * z.x, dlt * z.y));
        }
      }
    }
  } else {
    double g = 0.0;
    for (int s = 0; s < I.ns; ++s) {
      double v = 0.0;
      const double *cf = I.coef + ((int64_t)s * I.nn + t) * I.nrow;
      for (int r = 0; r < I.nrow; ++r) v += cf[r] * I.Ftab[(int64_t)r * I.nt + n];
      T *E = I.fields + ((int64_t)s * 6 + c) * I.F;
      const T old = E[idx];
      const T now = old - (T)(cev * v);
      E[idx] = now;
      if constexpr (ACC != ACC_NONE) {
        if (closing) {
          const double dlt = (double)old - (double)now;
          const int64_t base = (((int64_t)s * nf) * 3 + c) * I.F + idx;
          double re = 0.0;
          for (int kf = 0; kf < nf; ++kf) {
            const double2 Vk = acc_read<ACC>(I.vol, base + (int64_t)kf * 3 * I.F);
            const double2 Qt = I.Q[(int64_t)(n - 1) * nf + kf];
            re += Qt.x * Vk.x - Qt.y * Vk.y;
          }
          g += dlt * re;
        }
      }
    }
    if (closing) I.gedge[(int64_t)c * I.F + idx] += g;
  }
}

// transform of E at the receiver lattice nodes: one thread per (source, node)
template <typename T>
__global__ void k_rec_dft(int ns, int nn, const int *rn_c, const int64_t *rn_idx, const T *fields,
                          int64_t F, int nf, const double2 *zE, double2 *racc, const int *step) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns * nn) return;
  const int s = t / nn, node = t % nn;
  const int n = step[0];
  const double e = (double)fields[((int64_t)s * 6 + rn_c[node]) * F + rn_idx[node]];
  const double2 *z = zE + (int64_t)n * nf;
  double2 *a = racc + (int64_t)t * nf;
  for (int kf = 0; kf < nf; ++kf) {
    double2 v = a[kf];
    v.x = fma(e, z[kf].x, v.x);
    v.y = fma(e, z[kf].y, v.y);
    a[kf] = v;
  }
}

// receiver output: interpolate node transforms and scale per frequency
__global__ void k_rec_out(int ns, int nrows, int nn, int nf, const int *ptr, const int *node,
                          const double *w, const double2 *racc, const double2 *scale,
                          double2 *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns * nrows * nf) return;
  const int kf = t % nf, row = (t / nf) % nrows, s = t / (nf * nrows);
  double re = 0, im = 0;
  for (int e = ptr[row]; e < ptr[row + 1]; ++e) {
    const double2 a = racc[((int64_t)s * nn + node[e]) * nf + kf];
    re += w[e] * a.x;
    im += w[e] * a.y;
  }
  const double2 sc = scale[kf];
  out[t] = make_double2(re * sc.x - im * sc.y, re * sc.y + im * sc.x);
}

// gradient per cell from the 12 edges of the cell: with volume-weighted
// edge averaging, dV_e * d sigma_e / d sigma_c = V_c / 4 for every edge of
// the cell, so d phi / d ln rho_c = sigma_c V_c / 4 * sum_edges gacc * gscale
__global__ void k_grad_cells(int nx, int ny, int nz, int PX, int NY, int64_t F,
                             const double *gedge, const double *cellfac, double gscale,
                             double *grad, int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= nx) return;
  const int64_t plane = (int64_t)NY * PX;
  const int64_t q = (int64_t)k * plane + (int64_t)j * PX + i;
  const double *gx = gedge, *gy = gedge + F, *gz = gedge + 2 * F;
  const double sx = gx[q] + gx[q + PX] + gx[q + plane] + gx[q + plane + PX];
  const double sy = gy[q] + gy[q + 1] + gy[q + plane] + gy[q + plane + 1];
  const double sz = gz[q] + gz[q + 1] + gz[q + PX] + gz[q + PX + 1];
  const int64_t c = ((int64_t)k * ny + j) * nx + i;
  const double v = cellfac[c] * (sx + sy + sz) * gscale;
  grad[c] = accumulate ? grad[c] + v : v;
}

// normalised volume export: out[s][k][c][z][y][x] = V * scale_k; the
// (s, kf, c, z) planes are walked with a grid-stride loop over blockIdx.z
template <int ACC>
__global__ void k_vol_export(int ns, int nf, int NX, int NY, int NZ, int PX, int64_t F,
                             const void *vol, const double2 *scale, double2 *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= NX) return;
  const int total = ns * nf * 3 * NZ;
  for (int zc = blockIdx.z; zc < total; zc += gridDim.z) {
    const int k = zc % NZ;
    const int c = (zc / NZ) % 3;
    const int kf = (zc / (NZ * 3)) % nf;
    const int s = zc / (NZ * 3 * nf);
    const int64_t q = ((int64_t)k * NY + j) * PX + i;
    const double2 v = acc_read<ACC>(vol, (((int64_t)s * nf + kf) * 3 + c) * F + q);
    const double2 sc = scale[kf];
    out[(int64_t)zc * NY * NX + (int64_t)j * NX + i] =
        make_double2(v.x * sc.x - v.y * sc.y, v.x * sc.y + v.y * sc.x);
  }
}

__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

// ---------------------------------------------------------------------------
// device tables owned by the plan
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
};

struct Dev {
  int device = -1;
  uint64_t model_version = 0, basis_version = 0;
  std::vector<DevBuf> bufs;     // everything allocated for the tables
  // typed views
  void *ce[3] = {};
  void *ih[3] = {}, *ihd[3] = {};
  void *kn[3] = {}, *bn[3] = {}, *an[3] = {}, *kh[3] = {}, *bh[3] = {}, *ah[3] = {};
  double2 *zE = nullptr, *Q = nullptr;
  double *wavelet = nullptr, *basis = nullptr;
  int *src_s = nullptr, *src_c = nullptr, *src_toff = nullptr;
  int64_t *src_idx = nullptr;
  double *src_coef = nullptr;
  int *rn_c = nullptr;
  int64_t *rn_idx = nullptr;
  int *ri_ptr = nullptr, *ri_node = nullptr;
  double *ri_w = nullptr;
  double2 *fwd_scale = nullptr, *adj_scale_v = nullptr, *vol_scale = nullptr;
  // adjoint injection coefficients (rebuilt per call)
  double *at_coef = nullptr;
  double *cellfac = nullptr;
  double2 *eadj = nullptr;      // adjoint receiver transform when the caller passes none
  // graphs
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string exec_key;
  // sampled per-kernel timing
  std::vector<hipEvent_t> ev;
  double kstat_ms[4] = {0, 0, 0, 0};
  int kstat_n = 0;
  int sample_every = 0;
};

static Dev &D(Plan &p) {
  if (!p.dev) p.dev = new Dev();
  return *static_cast<Dev *>(p.dev);
}

static void *dalloc(Dev &d, size_t bytes) {
  void *ptr = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) fail(FWD_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  d.bufs.push_back({ptr, bytes});
  return ptr;
}

template <typename V>
static V *upload(Dev &d, const std::vector<V> &h) {
  V *p = static_cast<V *>(dalloc(d, h.size() * sizeof(V)));
  if (!h.empty()) HIP_CHECK(hipMemcpy(p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return p;
}

template <typename T>
static T *upload_as(Dev &d, const std::vector<double> &h) {
  std::vector<T> t(h.begin(), h.end());
  return upload(d, t);
}

static void free_tables(Dev &d) {
  for (auto &b : d.bufs) (void)hipFree(b.p);
  d.bufs.clear();
  if (d.exec) {
    (void)hipGraphExecDestroy(d.exec);
    d.exec = nullptr;
  }
  d.exec_key.clear();
}

void dev_release(Plan &p) {
  if (!p.dev) return;
  Dev &d = D(p);
  free_tables(d);
  if (d.cap) (void)hipStreamDestroy(d.cap);
  for (auto e : d.ev) (void)hipEventDestroy(e);
  delete &d;
  p.dev = nullptr;
}

template <typename T>
static void upload_model_tables(Plan &p, Dev &d) {
  for (int c = 0; c < 3; ++c) d.ce[c] = upload_as<T>(d, p.ce[c]);
  for (int a = 0; a < 3; ++a) {
    const Axis &ax = p.ax[a];
    std::vector<double> ih(ax.n), ihd(ax.n + 1);
    for (int i = 0; i < ax.n; ++i) ih[i] = 1.0 / ax.h[i];
    for (int i = 0; i <= ax.n; ++i) ihd[i] = 1.0 / ax.hd[i];
    d.ih[a] = upload_as<T>(d, ih);
    d.ihd[a] = upload_as<T>(d, ihd);
    d.kn[a] = upload_as<T>(d, ax.kinv_n);
    d.bn[a] = upload_as<T>(d, ax.b_n);
    d.an[a] = upload_as<T>(d, ax.a_n);
    d.kh[a] = upload_as<T>(d, ax.kinv_h);
    d.bh[a] = upload_as<T>(d, ax.b_h);
    d.ah[a] = upload_as<T>(d, ax.a_h);
  }
}

static void ensure_tables(Plan &p, hipStream_t stream) {
  if (!p.have_model) fail(FWD_ERR_STATE, "no model set");
  Dev &d = D(p);
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (d.model_version == p.model_version && d.basis_version == p.basis_version && d.device == dev)
    return;
  HIP_CHECK(hipStreamSynchronize(stream));
  free_tables(d);
  d.device = dev;
  if (!d.cap) HIP_CHECK(hipStreamCreateWithFlags(&d.cap, hipStreamNonBlocking));
  if (p.dtype == FWD_F64)
    upload_model_tables<double>(p, d);
  else
    upload_model_tables<float>(p, d);
  const int nf = p.nf();
  std::vector<double2> zE(p.zE.size());
  for (size_t q = 0; q < zE.size(); ++q) zE[q] = make_double2(p.zE[q].real(), p.zE[q].imag());
  d.zE = upload(d, zE);
  d.wavelet = upload(d, p.wavelet);
  // forward injection targets
  {
    std::vector<int> s, c, toff;
    std::vector<int64_t> idx;
    std::vector<double> coef;
    for (size_t t = 0; t < p.src_tg.size(); ++t) {
      s.push_back(p.src_tg[t].s);
      c.push_back(p.src_tg[t].c);
      idx.push_back(p.src_tg[t].idx);
      toff.push_back((int)t);
      coef.push_back(p.src_coef[t] * p.src_scale);
    }
    d.src_s = upload(d, s);
    d.src_c = upload(d, c);
    d.src_idx = upload(d, idx);
    d.src_toff = upload(d, toff);
    d.src_coef = upload(d, coef);
  }
  d.rn_c = upload(d, p.rn_c);
  d.rn_idx = upload(d, p.rn_idx);
  d.ri_ptr = upload(d, p.ri_ptr);
  d.ri_node = upload(d, p.ri_node);
  d.ri_w = upload(d, p.ri_w);
  std::vector<double2> sc(nf), vs(nf);
  for (int k = 0; k < nf; ++k) {
    const cplx v = p.norm[k] / p.src_scale;
    sc[k] = make_double2(v.real(), v.imag());
  }
  d.fwd_scale = upload(d, sc);
  d.vol_scale = d.fwd_scale;
  d.adj_scale_v = static_cast<double2 *>(dalloc(d, nf * sizeof(double2)));
  // adjoint injection coefficients [ns][node][2nf] (filled per adjoint call)
  {
    const int nn = (int)p.rn_c.size();
    d.at_coef = static_cast<double *>(dalloc(d, (size_t)p.ns * nn * 2 * nf * sizeof(double)));
    d.eadj = static_cast<double2 *>(dalloc(d, (size_t)p.ns * p.nr * p.ncomp * nf * sizeof(double2)));
  }
  // per-cell factor sigma V / 4 (zero for cells above the resistivity cap)
  {
    std::vector<double> cf((size_t)p.nx * p.ny * p.nz);
    for (int k = 0; k < p.nz; ++k)
      for (int j = 0; j < p.ny; ++j)
        for (int i = 0; i < p.nx; ++i) {
          const size_t c = ((size_t)k * p.ny + j) * p.nx + i;
          const double V = p.ax[0].h[i] * p.ax[1].h[j] * p.ax[2].h[k];
          cf[c] = p.capped[c] ? 0.0 : p.sigma[c] * V * 0.25;
        }
    d.cellfac = upload(d, cf);
  }
  if (p.have_basis) {
    d.basis = upload(d, p.basis);
    // Q_k^n = (Omega_k / w'_k) * norm_k * z_k^{n+1}: the discrete-time
    // gradient factor, the forward normalisation and the twiddle
    std::vector<double2> Q((size_t)p.nt * nf);
    for (int k = 0; k < nf; ++k) {
      const cplx f = p.Omega[k] / p.wprime[k] * p.norm[k];
      for (int n = 0; n < p.nt; ++n) {
        const cplx v = f * p.zE[(size_t)n * nf + k];
        Q[(size_t)n * nf + k] = make_double2(v.real(), v.imag());
      }
    }
    d.Q = upload(d, Q);
  }
  d.model_version = p.model_version;
  d.basis_version = p.basis_version;
}

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
struct WS {
  void *fields, *psi;
  double2 *racc;
  int *step;      // current step index
  int *flushed;   // last sample already added by a flush
  void *hist;
  double *gedge;
};

static size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

static WS carve(const Plan &p, void *ws) {
  WS w;
  char *b = static_cast<char *>(ws);
  w.fields = b;
  b += a256((size_t)p.ns * 6 * p.field_elems() * p.tsize());
  w.psi = b;
  b += a256((size_t)p.ns * p.psi_elems_per_source() * p.tsize());
  w.racc = reinterpret_cast<double2 *>(b);
  b += a256((size_t)p.ns * p.rn_c.size() * p.nf() * 16);
  w.step = reinterpret_cast<int *>(b);
  w.flushed = w.step + 1;
  b += 256;
  w.hist = b;
  b += a256((size_t)p.ns * p.hist_elems_per_source() * p.tsize());
  w.gedge = reinterpret_cast<double *>(b);
  return w;
}

// ---------------------------------------------------------------------------
// one step = four launches
// ---------------------------------------------------------------------------
struct Launch {
  int mode;       // FWD_MODE_*
  bool volume;    // forward: accumulate the volume transform
  int block_x, block_y;
};

template <typename T>
static StepArgs<T> make_args(Plan &p, Dev &d, const WS &w, void *vol, bool adj) {
  StepArgs<T> A{};
  A.nx = p.nx;
  A.ny = p.ny;
  A.nz = p.nz;
  A.npml = p.npml;
  A.PX = p.PX;
  A.NY = p.NY;
  A.NZ = p.NZ;
  A.ns = p.ns;
  A.F = p.field_elems();
  A.psi_src = p.psi_elems_per_source();
  A.fields = static_cast<T *>(w.fields);
  A.psi = static_cast<T *>(w.psi);
  for (int c = 0; c < 3; ++c) A.ce[c] = static_cast<const T *>(d.ce[c]);
  for (int a = 0; a < 3; ++a) {
    A.ax[a].ih = static_cast<const T *>(d.ih[a]);
    A.ax[a].ihd = static_cast<const T *>(d.ihd[a]);
    A.ax[a].kn = static_cast<const T *>(d.kn[a]);
    A.ax[a].bn = static_cast<const T *>(d.bn[a]);
    A.ax[a].an = static_cast<const T *>(d.an[a]);
    A.ax[a].kh = static_cast<const T *>(d.kh[a]);
    A.ax[a].bh = static_cast<const T *>(d.bh[a]);
    A.ax[a].ah = static_cast<const T *>(d.ah[a]);
  }
  A.dtmu = (T)(p.dt / kMu0);
  A.step = w.step;
  A.step_w = w.step;
  A.nbx = (p.NX + p.bx - 1) / p.bx;
  A.nby = (p.NY + p.by - 1) / p.by;
  A.nbz = p.NZ;
  A.nblocks = A.nbx * A.nby * A.nbz;
  A.xcd = p.xcd;
  A.nf = p.nf();
  A.zE = d.zE;
  A.vol = vol;
  A.Q = d.Q;
  A.gedge = adj ? w.gedge : nullptr;
  A.hist = static_cast<T *>(w.hist);
  A.hist_src = p.hist_elems_per_source();
  A.flushed = w.flushed;
  return A;
}

template <typename T, int KB>
static void launch_e_kb(const StepArgs<T> &A, int acc, bool adj, bool flush, dim3 grid, dim3 block,
                        hipStream_t st) {
#define FWD_LAUNCH(ACCV, ADJV)                                                                 \
  do {                                                                                         \
    if (flush) hipLaunchKernelGGL((k_flush<T, ACCV, ADJV, KB>), grid, block, 0, st, A);        \
    else hipLaunchKernelGGL((k_update_e<T, ACCV, ADJV, KB>), grid, block, 0, st, A);           \
  } while (0)
  if (!A.vol) {
    if (!flush) hipLaunchKernelGGL((k_update_e<T, ACC_NONE, false, 1>), grid, block, 0, st, A);
    return;
  }
  switch (acc) {
    case FWD_ACC_F64:
      if (adj) FWD_LAUNCH(ACC_F64, true); else FWD_LAUNCH(ACC_F64, false);
      break;
    case FWD_ACC_KAHAN:
      if (adj) FWD_LAUNCH(ACC_KAHAN, true); else FWD_LAUNCH(ACC_KAHAN, false);
      break;
    default:
      if (adj) FWD_LAUNCH(ACC_F32, true); else FWD_LAUNCH(ACC_F32, false);
  }
#undef FWD_LAUNCH
}

// E update (flush = false) or the flush of an incomplete transform block
template <typename T>
static void launch_e(const StepArgs<T> &A, int kb, int acc, bool adj, bool flush, dim3 grid,
                     dim3 block, hipStream_t st) {
  switch (kb) {
    case 1: launch_e_kb<T, 1>(A, acc, adj, flush, grid, block, st); break;
    case 2: launch_e_kb<T, 2>(A, acc, adj, flush, grid, block, st); break;
    case 4: launch_e_kb<T, 4>(A, acc, adj, flush, grid, block, st); break;
    default: launch_e_kb<T, 8>(A, acc, adj, flush, grid, block, st);
  }
}

template <typename T, int KB>
static void launch_inject_kb(const InjArgs<T> &I, int acc, bool adj, hipStream_t st) {
  const dim3 grid((I.ntg + 63) / 64), block(64);
#define FWD_INJ(ACCV)                                                                         \
  do {                                                                                        \
    if (adj) hipLaunchKernelGGL((k_inject<T, ACCV, true, KB>), grid, block, 0, st, I);        \
    else hipLaunchKernelGGL((k_inject<T, ACCV, false, KB>), grid, block, 0, st, I);           \
  } while (0)
  switch (acc) {
    case FWD_ACC_F64: FWD_INJ(ACC_F64); break;
    case FWD_ACC_KAHAN: FWD_INJ(ACC_KAHAN); break;
    case FWD_ACC_F32: FWD_INJ(ACC_F32); break;
    default: hipLaunchKernelGGL((k_inject<T, ACC_NONE, false, 1>), grid, block, 0, st, I);
  }
#undef FWD_INJ
}

template <typename T>
static void launch_inject(const InjArgs<T> &I, int kb, int acc, bool adj, hipStream_t st) {
  switch (kb) {
    case 1: launch_inject_kb<T, 1>(I, acc, adj, st); break;
    case 2: launch_inject_kb<T, 2>(I, acc, adj, st); break;
    case 4: launch_inject_kb<T, 4>(I, acc, adj, st); break;
    default: launch_inject_kb<T, 8>(I, acc, adj, st);
  }
}

// enqueue one step; if ev != nullptr, record ev[0..4] around the 4 kernels
template <typename T>
static void enqueue_step(Plan &p, Dev &d, const WS &w, void *vol, bool adj, hipStream_t st,
                         hipEvent_t *ev) {
  StepArgs<T> A = make_args<T>(p, d, w, vol, adj);
  const dim3 block(p.bx, p.by), grid(A.nblocks);
  const int64_t F = A.F;
  T *fields = static_cast<T *>(w.fields);
  const int nn = (int)p.rn_c.size();
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((k_update_h<T>), grid, block, 0, st, A);
  if (ev) (void)hipEventRecord(ev[1], st);
  {
    InjArgs<T> I{};
    I.nt = p.nt;
    I.ns = p.ns;
    I.nn = nn;
    I.nf = p.nf();
    I.fields = fields;
    I.F = F;
    I.ce0 = static_cast<const T *>(d.ce[0]);
    I.ce1 = static_cast<const T *>(d.ce[1]);
    I.ce2 = static_cast<const T *>(d.ce[2]);
    I.step = w.step;
    I.flushed = w.flushed;
    I.vol = vol;
    I.zE = d.zE;
    I.Q = d.Q;
    I.gedge = adj ? w.gedge : nullptr;
    if (!adj) {
      I.ntg = (int)p.src_tg.size();
      I.nrow = 1;
      I.tg_s = d.src_s;
      I.tg_c = d.src_c;
      I.tg_toff = d.src_toff;
      I.tg_idx = d.src_idx;
      I.coef = d.src_coef;
      I.Ftab = d.wavelet;
    } else {
      I.ntg = nn;
      I.nrow = 2 * p.nf();
      I.tg_c = d.rn_c;
      I.tg_idx = d.rn_idx;
      I.coef = d.at_coef;
      I.Ftab = d.basis;
    }
    launch_inject<T>(I, p.kb, vol ? p.acc : -1, adj, st);
  }
  if (ev) (void)hipEventRecord(ev[2], st);
  launch_e<T>(A, p.kb, p.acc, adj, false, grid, block, st);
  if (ev) (void)hipEventRecord(ev[3], st);
  const int nrt = p.ns * nn;
  hipLaunchKernelGGL((k_rec_dft<T>), dim3((nrt + 63) / 64), dim3(64), 0, st, p.ns, nn, d.rn_c,
                     d.rn_idx, (const T *)fields, F, p.nf(), d.zE, w.racc, (const int *)w.step);
  if (ev) (void)hipEventRecord(ev[4], st);
}

template <typename T>
static void flush_t(Plan &p, Dev &d, const WS &w, void *vol, bool adj, hipStream_t st) {
  if (p.kb == 1 || !vol) return;
  StepArgs<T> A = make_args<T>(p, d, w, vol, adj);
  launch_e<T>(A, p.kb, p.acc, adj, true, dim3(A.nblocks), dim3(p.bx, p.by), st);
  hipLaunchKernelGGL(k_set_flushed, dim3(1), dim3(64), 0, st, w.flushed, (const int *)w.step);
  HIP_CHECK(hipGetLastError());
}

static void flush_any(Plan &p, Dev &d, const WS &w, void *vol, bool adj, hipStream_t st) {
  if (p.dtype == FWD_F64)
    flush_t<double>(p, d, w, vol, adj, st);
  else
    flush_t<float>(p, d, w, vol, adj, st);
}

template <typename T>
static void run_steps_t(Plan &p, Dev &d, const WS &w, void *vol, bool adj, int nsteps,
                        hipStream_t st) {
  const int K = p.graph_steps;
  const int sample = d.sample_every;
  // eager launches of m steps, each bracketed by events if asked
  auto eager = [&](int m, bool timed) {
    for (int t = 0; t < m; ++t) {
      hipEvent_t *ev = nullptr;
      if (timed) {
        const size_t need = (size_t)(d.kstat_n + 1) * 5;
        while (d.ev.size() < need) {
          hipEvent_t e;
          HIP_CHECK(hipEventCreate(&e));
          d.ev.push_back(e);
        }
        ev = &d.ev[(size_t)d.kstat_n * 5];
        d.kstat_n++;
      }
      enqueue_step<T>(p, d, w, vol, adj, st, ev);
    }
    HIP_CHECK(hipGetLastError());
  };
  if (K <= 1 || nsteps < K) {
    for (int t = 0; t < nsteps; ++t) eager(1, sample > 0 && t % sample == 0);
    return;
  }
  // graph of K steps, captured on a private stream and replayed on st
  char key[256];
  snprintf(key, sizeof key, "%p/%p/%d/%d/%d/%d/%d/%d/%llu/%llu", w.fields, vol, (int)adj, K, p.bx,
           p.by, p.xcd, p.kb, (unsigned long long)p.model_version,
           (unsigned long long)p.basis_version);
  if (!d.exec || d.exec_key != key) {
    if (d.exec) {
      HIP_CHECK(hipGraphExecDestroy(d.exec));
      d.exec = nullptr;
    }
    hipGraph_t g;
    HIP_CHECK(hipStreamBeginCapture(d.cap, hipStreamCaptureModeRelaxed));
    for (int t = 0; t < K; ++t) enqueue_step<T>(p, d, w, vol, adj, d.cap, nullptr);
    HIP_CHECK(hipStreamEndCapture(d.cap, &g));
    HIP_CHECK(hipGraphInstantiate(&d.exec, g, nullptr, nullptr, 0));
    HIP_CHECK(hipGraphDestroy(g));
    d.exec_key = key;
  }
  // with sampling on, one chunk in every max(1, sample/K) runs eagerly and
  // times each of its steps (all phases of the transform block); all others
  // replay the graph
  const int every = sample > 0 ? std::max(1, sample / K) : 0;
  int done = 0, chunk = 0;
  while (nsteps - done >= K) {
    if (every && chunk % every == 0) {
      eager(K, true);
    } else {
      HIP_CHECK(hipGraphLaunch(d.exec, st));
    }
    done += K;
    ++chunk;
  }
  eager(nsteps - done, false);
}

static void run_steps_any(Plan &p, Dev &d, const WS &w, void *vol, bool adj, int nsteps,
                          hipStream_t st) {
  if (p.dtype == FWD_F64)
    run_steps_t<double>(p, d, w, vol, adj, nsteps, st);
  else
    run_steps_t<float>(p, d, w, vol, adj, nsteps, st);
}

static void collect_kernel_stats(Dev &d) {
  double tot[4] = {0, 0, 0, 0};
  for (int s = 0; s < d.kstat_n; ++s) {
    hipEvent_t *ev = &d.ev[(size_t)s * 5];
    for (int k = 0; k < 4; ++k) {
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      tot[k] += ms;
    }
  }
  for (int k = 0; k < 4; ++k) d.kstat_ms[k] = d.kstat_n ? tot[k] / d.kstat_n : 0.0;
}

static void zero_state(Plan &p, const WS &w, void *ws, void *vol, int mode, hipStream_t st) {
  HIP_CHECK(hipMemsetAsync(ws, 0, p.workspace_bytes(mode), st));
  if (vol && mode == FWD_MODE_FORWARD) HIP_CHECK(hipMemsetAsync(vol, 0, p.volume_bytes(), st));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, w.step, -1);
  HIP_CHECK(hipGetLastError());
}

static void check_sizes(Plan &p, size_t ws_bytes, int mode, void *vol, size_t vol_bytes) {
  if (ws_bytes < p.workspace_bytes(mode)) fail(FWD_ERR_INVALID_ARG, "workspace too small");
  if (vol && vol_bytes < p.volume_bytes()) fail(FWD_ERR_INVALID_ARG, "volume buffer too small");
}

static void check_finite(const double2 *dptr, size_t n, hipStream_t st) {
  std::vector<double2> h(n);
  HIP_CHECK(hipMemcpyAsync(h.data(), dptr, n * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (auto &v : h)
    if (!std::isfinite(v.x) || !std::isfinite(v.y))
      fail(FWD_ERR_NONFINITE, "non-finite field: unstable run (dt above the CFL bound?)");
}

// ---------------------------------------------------------------------------
// entry points used by the C ABI
// ---------------------------------------------------------------------------
void dev_run_begin(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  check_sizes(p, ws_bytes, FWD_MODE_FORWARD, vol, vol_bytes);
  ensure_tables(p, st);
  zero_state(p, carve(p, ws), ws, vol, FWD_MODE_FORWARD, st);
}

void dev_run_steps(Plan &p, void *ws, void *vol, int nsteps, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  ensure_tables(p, st);
  if (nsteps < 0) fail(FWD_ERR_INVALID_ARG, "nsteps < 0");
  Dev &d = D(p);
  run_steps_any(p, d, carve(p, ws), vol, false, nsteps, st);
}

void dev_run_receivers(Plan &p, void *ws, double *E_rec, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  ensure_tables(p, st);
  Dev &d = D(p);
  WS w = carve(p, ws);
  const int nrows = p.nr * p.ncomp, nn = (int)p.rn_c.size(), n = p.ns * nrows * p.nf();
  hipLaunchKernelGGL(k_rec_out, dim3((n + 127) / 128), dim3(128), 0, st, p.ns, nrows, nn, p.nf(),
                     d.ri_ptr, d.ri_node, d.ri_w, w.racc, d.fwd_scale,
                     reinterpret_cast<double2 *>(E_rec));
  HIP_CHECK(hipGetLastError());
}

void dev_run_flush(Plan &p, void *ws, void *vol, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  ensure_tables(p, st);
  flush_any(p, D(p), carve(p, ws), vol, false, st);
}

void dev_forward(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes, double *E_rec,
                 void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  dev_run_begin(p, ws, ws_bytes, vol, vol_bytes, stream);
  Dev &d = D(p);
  d.kstat_n = 0;
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipEventRecord(e0, st));
  run_steps_any(p, d, carve(p, ws), vol, false, p.nt, st);
  flush_any(p, d, carve(p, ws), vol, false, st);
  HIP_CHECK(hipEventRecord(e1, st));
  dev_run_receivers(p, ws, E_rec, stream);
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p.last_ms = ms;
  p.last_steps = p.nt;
  collect_kernel_stats(d);
  check_finite(reinterpret_cast<double2 *>(E_rec), (size_t)p.ns * p.nr * p.ncomp * p.nf(), st);
}

void dev_checkpoint(Plan &p, const void *ws, const void *vol, void *snap, int save, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t sb = p.state_bytes();
  char *sn = static_cast<char *>(snap);
  if (save) {
    HIP_CHECK(hipMemcpyAsync(sn, ws, sb, hipMemcpyDeviceToDevice, st));
    if (vol) HIP_CHECK(hipMemcpyAsync(sn + sb, vol, p.volume_bytes(), hipMemcpyDeviceToDevice, st));
  } else {
    HIP_CHECK(hipMemcpyAsync(const_cast<void *>(ws), sn, sb, hipMemcpyDeviceToDevice, st));
    if (vol)
      HIP_CHECK(hipMemcpyAsync(const_cast<void *>(vol), sn + sb, p.volume_bytes(),
                               hipMemcpyDeviceToDevice, st));
  }
}

void dev_volume_export(Plan &p, const void *vol, double *out, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  ensure_tables(p, st);
  Dev &d = D(p);
  if (p.NY > 65535) fail(FWD_ERR_UNSUPPORTED, "volume export: ny too large");
  const dim3 block(64), grid((p.NX + 63) / 64, p.NY, std::min(p.ns * p.nf() * 3 * p.NZ, 4096));
  double2 *o = reinterpret_cast<double2 *>(out);
  switch (p.acc) {
    case FWD_ACC_F64:
      hipLaunchKernelGGL((k_vol_export<ACC_F64>), grid, block, 0, st, p.ns, p.nf(), p.NX, p.NY, p.NZ,
                         p.PX, p.field_elems(), vol, d.vol_scale, o);
      break;
    case FWD_ACC_KAHAN:
      hipLaunchKernelGGL((k_vol_export<ACC_KAHAN>), grid, block, 0, st, p.ns, p.nf(), p.NX, p.NY,
                         p.NZ, p.PX, p.field_elems(), vol, d.vol_scale, o);
      break;
    default:
      hipLaunchKernelGGL((k_vol_export<ACC_F32>), grid, block, 0, st, p.ns, p.nf(), p.NX, p.NY, p.NZ,
                         p.PX, p.field_elems(), vol, d.vol_scale, o);
  }
  HIP_CHECK(hipGetLastError());
}

void dev_adjoint(Plan &p, void *ws, size_t ws_bytes, const void *vol, const double *resid,
                 double *grad, int accumulate, double *E_adj, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!p.have_basis) fail(FWD_ERR_BASIS, "build the basis functions first (fwd_basis_build)");
  if (!vol) fail(FWD_ERR_INVALID_ARG, "adjoint needs the forward volume transform");
  check_sizes(p, ws_bytes, FWD_MODE_ADJOINT, const_cast<void *>(vol), p.volume_bytes());
  ensure_tables(p, st);
  Dev &d = D(p);
  WS w = carve(p, ws);
  // adjoint coefficients on the host (small): residual -> spectrum -> nodes
  const size_t nres = (size_t)p.ns * p.nr * p.ncomp * p.nf();
  std::vector<double> rh(2 * nres);
  HIP_CHECK(hipMemcpyAsync(rh.data(), resid, rh.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<double> T;
  double adj_scale = 1.0;
  adjoint_coefficients(p, rh.data(), T, adj_scale);
  HIP_CHECK(hipMemcpyAsync(d.at_coef, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<double2> as(p.nf(), make_double2(1.0 / adj_scale, 0.0));
  HIP_CHECK(hipMemcpyAsync(d.adj_scale_v, as.data(), as.size() * sizeof(double2),
                           hipMemcpyHostToDevice, st));
  zero_state(p, w, ws, nullptr, FWD_MODE_ADJOINT, st);
  d.kstat_n = 0;
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipEventRecord(e0, st));
  run_steps_any(p, d, w, const_cast<void *>(vol), true, p.nt, st);
  flush_any(p, d, w, const_cast<void *>(vol), true, st);
  HIP_CHECK(hipEventRecord(e1, st));
  // gradient on cells
  const double gscale = 1.0 / (p.src_scale * adj_scale);
  hipLaunchKernelGGL(k_grad_cells, dim3((p.nx + 127) / 128, p.ny, p.nz), dim3(128), 0, st, p.nx,
                     p.ny, p.nz, p.PX, p.NY, p.field_elems(), w.gedge, d.cellfac, gscale, grad,
                     accumulate);
  HIP_CHECK(hipGetLastError());
  const int nrows = p.nr * p.ncomp, nn = (int)p.rn_c.size(), n = p.ns * nrows * p.nf();
  double2 *dst = E_adj ? reinterpret_cast<double2 *>(E_adj) : d.eadj;
  hipLaunchKernelGGL(k_rec_out, dim3((n + 127) / 128), dim3(128), 0, st, p.ns, nrows, nn, p.nf(),
                     d.ri_ptr, d.ri_node, d.ri_w, w.racc, d.adj_scale_v, dst);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p.last_ms = ms;
  p.last_steps = p.nt;
  collect_kernel_stats(d);
  check_finite(dst, (size_t)n, st);
}

// ---------------------------------------------------------------------------
// autotuner: time each (block shape, XCD remap) candidate on the real buffers
// ---------------------------------------------------------------------------
double dev_autotune(Plan &p, void *ws, size_t ws_bytes, void *vol, size_t vol_bytes, int mode,
                    int steps, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool adj = mode == FWD_MODE_ADJOINT;
  if (adj && (!p.have_basis || !vol)) fail(FWD_ERR_STATE, "adjoint tuning needs basis and volume");
  check_sizes(p, ws_bytes, mode, vol, vol_bytes);
  ensure_tables(p, st);
  Dev &d = D(p);
  WS w = carve(p, ws);
  const int cand[][2] = {{64, 4}, {64, 2}, {128, 2}, {128, 1}, {256, 1}, {64, 1}};
  const int save_bx = p.bx, save_by = p.by, save_xcd = p.xcd, save_sample = d.sample_every;
  d.sample_every = 0;
  double best = 1e300;
  int bbx = save_bx, bby = save_by, bxcd = save_xcd;
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  for (auto &c : cand) {
    for (int xc = 0; xc <= 1; ++xc) {
      p.bx = c[0];
      p.by = c[1];
      p.xcd = xc;
      zero_state(p, w, ws, adj ? nullptr : vol, mode, st);
      run_steps_any(p, d, w, vol, adj, 4, st);   // warm-up (graph capture)
      HIP_CHECK(hipEventRecord(e0, st));
      run_steps_any(p, d, w, vol, adj, steps, st);
      HIP_CHECK(hipEventRecord(e1, st));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      const double per = ms / steps;
      if (per < best) {
        best = per;
        bbx = c[0];
        bby = c[1];
        bxcd = xc;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p.bx = bbx;
  p.by = bby;
  p.xcd = bxcd;
  d.sample_every = save_sample;
  return best;
}

// option plumbing for the sampled timing lives with the device state
void dev_set_sampling(Plan &p, int every) { D(p).sample_every = every; }
int dev_get_sampling(Plan &p) { return p.dev ? D(p).sample_every : 0; }
void dev_kernel_stats(Plan &p, double *ms4, int *count) {
  if (!p.dev) {
    for (int k = 0; k < 4; ++k) ms4[k] = 0;
    *count = 0;
    return;
  }
  Dev &d = D(p);
  for (int k = 0; k < 4; ++k) ms4[k] = d.kstat_ms[k];
  *count = d.kstat_n;
}

}  // namespace fwdem
