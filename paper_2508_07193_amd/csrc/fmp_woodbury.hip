// Index-block subdomains with the low-rank boundary correction (FP64).
//
// The paper's own subdomain (Sec. III-A): the unknowns whose indices fall in
// a block of the global grid, for half points and nodes alike, extended by
// the overlap (0 allowed).  Its operator I + alpha M is built from the
// compact forward difference D^f (n x n, the node past the block's end taken
// as zero), whose SVD D^f = U S V^T has a closed form with
//     theta_m = (2m - 1) pi / (2n + 1),  sigma_m = 2 sin(theta_m / 2),
//     V[i][m] = c cos(theta_m (i + 1/2)),  U[i][m] = -c sin(theta_m (i + 1)),
//     c = 2 / sqrt(2n + 1),
// so the transform G (U^T along a component's own axis, V^T along its node
// axes, eq. (9)) turns it into the 3x3 blocks B_ijk of eq. (12), solved in
// closed form per wavenumber: exact_solve of Algorithm 1.
//
// The restriction of the global operator to the block differs from
// I + alpha M on the block's low faces only (Step 4): alpha times delta, the
// number of node axes along which the slot lies on the low face.  With Q the
// selection of those 6n^2 - 3n slots and W = alpha diag(delta), Woodbury
// gives the block's exact inverse as
//     E = exact_solve(R);  E -= exact_solve(Q C^{-1} Q^T E),
//     C = W^{-1} + Q^T (I + alpha M)^{-1} Q,
// Algorithm 1's main body.  A box that starts at a global PEC wall holds
// that wall's nodes; their slots are constrained to zero by giving them
// W^{-1} = 0 (the limit of an infinite weight), which leaves the restricted
// system on the other unknowns exact.
//
// Per apply (all boxes at once, staging W_E and W_C of full box arrays):
//   A, B, C      exact_solve(S^gamma r) -> W_E           (three passes)
//   qgather      g = Q^T E                                (per box)
//   cgemv        h = C^{-1} g                             (boxes sharing C^{-1} together)
//   qscatter     W_C = Q h
//   A, B, C      z = S^0T (E - exact_solve(W_C))          (owned unknowns)
// Setup builds every distinct C^{-1} (box shape, wall pattern, alpha) on the
// device: the columns A0^{-1} Q from batched exact solves of unit vectors,
// C from their boundary rows plus W^{-1}, then an in-place blocked
// Gauss-Jordan inversion (C is symmetric positive definite, no pivoting).
//
// Contractions follow the vector-ALU passes of the PEC boxes: one pencil per
// lane in registers, table rows as scalar operands, but dense (the compact
// bases have no even/odd symmetry to halve them).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>

#include "fmp_common.h"
#include "fmp_ctx.h"

namespace fmp {
namespace {

constexpr int kIBT = 128;       // threads of passes A / C
constexpr int kIBClasses[] = {8, 16, 24, 32, 34, 48};
constexpr int kNumIBClasses = sizeof(kIBClasses) / sizeof(kIBClasses[0]);

template <int NP>
__device__ __forceinline__ double dot_row(const double* __restrict__ row, const double (&v)[NP]) {
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int j = 0; j + 1 < NP; j += 2) {
    a0 = __builtin_fma(row[j], v[j], a0);
    a1 = __builtin_fma(row[j + 1], v[j + 1], a1);
  }
  if (NP & 1) a0 = __builtin_fma(row[NP - 1], v[NP - 1], a0);
  return a0 + a1;
}

__device__ __forceinline__ const double* ib_table(const double* tab, const BoxDev& B, int axis,
                                                  int kind) {
  return tab + B.ibt[axis] + (long long)kind * kIT * kIT;
}
// forward table of component q along axis a: U^T on its own axis, V^T elsewhere
__device__ __forceinline__ const double* ib_fwd(const double* tab, const BoxDev& B, int q, int a) {
  return ib_table(tab, B, a, q == a ? 0 : 2);
}
__device__ __forceinline__ const double* ib_inv(const double* tab, const BoxDev& B, int q, int a) {
  return ib_table(tab, B, a, q == a ? 1 : 3);
}

template <int NP>
constexpr int ib_zs() {
  return kIBT / NP > 0 ? kIBT / NP : 1;
}

// ---------------------------------------------------------------- pass A
// Work item (box, component, first plane of a slab of ib_zs planes).
// Win may be W itself (a slab is read whole before it is written back).
template <int NP>
__global__ __launch_bounds__(kIBT) void k_ib_a(const double* __restrict__ r, const double* Win,
                                               double* W,
                                               const BoxDev* __restrict__ boxes,
                                               const DomainDev* __restrict__ doms,
                                               const int4* __restrict__ work,
                                               const double* __restrict__ tab) {
  constexpr int ZS = ib_zs<NP>();
  __shared__ double buf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int plane = nx * ny;
  const int tot = nzs * plane;
  const int t = threadIdx.x;
  if (Win) {                                      // staged box arrays
    const double* src = Win + B.w_off + (long long)q * B.vol + (long long)z0 * plane;
    for (int e = t; e < tot; e += kIBT) buf[e] = src[e];
  } else {                                        // S^gamma r, wall slots 0
    const DomainDev& D = doms[B.dom];
    const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
    for (int e = t; e < tot; e += kIBT) {
      const int zl = e / plane, rem = e - zl * plane, y = rem / nx, x = rem - y * nx;
      const int gx = B.bx0 + x, gy = B.by0 + y, gz = B.bz0 + z0 + zl;
      const bool wall = (q != 0 && gx == 0) || (q != 1 && gy == 0) || (q != 2 && gz == 0);
      buf[e] = wall ? 0.0 : src[((long long)gz * D.ny + gy) * D.nx + gx];
    }
  }
  __syncthreads();
  {                                               // x, one row per lane, in place
    const double* T = ib_fwd(tab, B, q, 0);
    for (int row = t; row < nzs * ny; row += kIBT) {
      double v[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) v[l] = l < nx ? buf[row * nx + l] : 0.0;
#pragma unroll 1
      for (int p = 0; p < nx; ++p) buf[row * nx + p] = dot_row<NP>(T + p * kIT, v);
    }
  }
  __syncthreads();
  {                                               // y, one column per lane, to W
    const double* T = ib_fwd(tab, B, q, 1);
    for (int col = t; col < nzs * nx; col += kIBT) {
      const int zl = col / nx, x = col - zl * nx;
      double v[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) v[m] = m < ny ? buf[zl * plane + m * nx + x] : 0.0;
      double* dst = W + B.w_off + (long long)q * B.vol + (long long)(z0 + zl) * plane + x;
#pragma unroll 1
      for (int p = 0; p < ny; ++p) dst[p * nx] = dot_row<NP>(T + p * kIT, v);
    }
  }
}

// ---------------------------------------------------------------- pass B
// Work item (box, first of 64 (x, y) columns); one wave per component.
template <int NP>
__global__ __launch_bounds__(192) void k_ib_b(double* __restrict__ W,
                                              const BoxDev* __restrict__ boxes,
                                              const int4* __restrict__ work,
                                              const double* __restrict__ tab) {
  __shared__ double ex[3][NP][64];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int plane = nx * ny;
  const int c = wk.y + lane;
  const bool active = c < plane;
  double* col = W + B.w_off + (long long)q * B.vol + (active ? c : 0);
  double v[NP];
#pragma unroll
  for (int l = 0; l < NP; ++l) v[l] = col[(long long)min(l, nz - 1) * plane];
#pragma unroll
  for (int l = 0; l < NP; ++l) v[l] = l < nz ? v[l] : 0.0;
  {
    const double* T = ib_fwd(tab, B, q, 2);
#pragma unroll 1
    for (int rr = 0; rr < nz; ++rr) ex[q][rr][lane] = dot_row<NP>(T + rr * kIT, v);
  }
  __syncthreads();
  // e = (r + alpha s (s.r)) / (1 + alpha |s|^2) with the compact sigmas
  const int yy = active ? c / nx : 0;
  const int xx = active ? c - yy * nx : 0;
  const double sx = ib_table(tab, B, 0, 4)[xx];
  const double sy = ib_table(tab, B, 1, 4)[yy];
  const double* sz = ib_table(tab, B, 2, 4);
  const double alpha = B.alpha;
  for (int rr = q; rr < nz; rr += 3) {
    const double s3 = sz[rr];
    const double a = ex[0][rr][lane], b = ex[1][rr][lane], d = ex[2][rr][lane];
    const double dot = __builtin_fma(sx, a, __builtin_fma(sy, b, s3 * d));
    const double den = __builtin_fma(alpha, __builtin_fma(s3, s3, __builtin_fma(sx, sx, sy * sy)), 1.0);
    const double inv = 1.0 / den;
    ex[0][rr][lane] = __builtin_fma(alpha * sx, dot, a) * inv;
    ex[1][rr][lane] = __builtin_fma(alpha * sy, dot, b) * inv;
    ex[2][rr][lane] = __builtin_fma(alpha * s3, dot, d) * inv;
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < NP; ++rr) v[rr] = rr < nz ? ex[q][rr][lane] : 0.0;
  {
    const double* T = ib_inv(tab, B, q, 2);
#pragma unroll 1
    for (int l = 0; l < nz; ++l) {
      const double o = dot_row<NP>(T + l * kIT, v);
      if (active) col[(long long)l * plane] = o;
    }
  }
}

// ---------------------------------------------------------------- pass C
// Work item as pass A.  z == nullptr: the full box arrays go to Wdst (which
// may be Wsrc).  Otherwise z = E - (result) on the owned unknowns, wall slots 0.
template <int NP>
__global__ __launch_bounds__(kIBT) void k_ib_c(const double* Wsrc, double* Wdst,
                                               const double* __restrict__ E,
                                               double* __restrict__ z,
                                               const BoxDev* __restrict__ boxes,
                                               const DomainDev* __restrict__ doms,
                                               const int4* __restrict__ work,
                                               const double* __restrict__ tab) {
  constexpr int ZS = ib_zs<NP>();
  __shared__ double buf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int plane = nx * ny;
  const int tot = nzs * plane;
  const int t = threadIdx.x;
  const long long base = B.w_off + (long long)q * B.vol + (long long)z0 * plane;
  for (int e = t; e < tot; e += kIBT) buf[e] = Wsrc[base + e];
  __syncthreads();
  {                                               // y inverse, one column per lane
    const double* T = ib_inv(tab, B, q, 1);
    for (int col = t; col < nzs * nx; col += kIBT) {
      const int zl = col / nx, x = col - zl * nx;
      double v[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) v[m] = m < ny ? buf[zl * plane + m * nx + x] : 0.0;
#pragma unroll 1
      for (int j = 0; j < ny; ++j) buf[zl * plane + j * nx + x] = dot_row<NP>(T + j * kIT, v);
    }
  }
  __syncthreads();
  {                                               // x inverse, one row per lane
    const double* T = ib_inv(tab, B, q, 0);
    for (int row = t; row < nzs * ny; row += kIBT) {
      double v[NP];
#pragma unroll
      for (int l = 0; l < NP; ++l) v[l] = l < nx ? buf[row * nx + l] : 0.0;
#pragma unroll 1
      for (int i = 0; i < nx; ++i) buf[row * nx + i] = dot_row<NP>(T + i * kIT, v);
    }
  }
  __syncthreads();
  if (!z) {
    for (int e = t; e < tot; e += kIBT) Wdst[base + e] = buf[e];
    return;
  }
  // S^0T: the owned part of the slab
  const int lz0 = max(z0, B.oz0 - B.bz0), lz1 = min(z0 + nzs, B.oz0 - B.bz0 + B.sz);
  if (lz1 <= lz0) return;
  const int ly0 = B.oy0 - B.by0, lx0 = B.ox0 - B.bx0;
  const int oplane = B.sx * B.sy;
  const int otot = (lz1 - lz0) * oplane;
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  for (int e = t; e < otot; e += kIBT) {
    const int zl = e / oplane, rem = e - zl * oplane, y = rem / B.sx, x = rem - y * B.sx;
    const int bz = lz0 + zl, by = ly0 + y, bx = lx0 + x;
    const int gx = B.bx0 + bx, gy = B.by0 + by, gz = B.bz0 + bz;
    const bool wall = (q != 0 && gx == 0) || (q != 1 && gy == 0) || (q != 2 && gz == 0);
    const int bi = (bz - z0) * plane + by * nx + bx;
    const long long wi = B.w_off + (long long)q * B.vol + (long long)bz * plane + by * nx + bx;
    dst[((long long)gz * D.ny + gy) * D.nx + gx] = wall ? 0.0 : E[wi] - buf[bi];
  }
}

// ---------------------------------------------------------------- boundary slots
// g[box][j] = W[box][Q_j]   (one block row per box)
__global__ __launch_bounds__(256) void k_ib_qgather(const double* __restrict__ W,
                                                    const BoxDev* __restrict__ boxes,
                                                    const int* __restrict__ qidx,
                                                    double* __restrict__ g) {
  const BoxDev& B = boxes[blockIdx.y];
  for (int j = blockIdx.x * 256 + threadIdx.x; j < B.m; j += gridDim.x * 256)
    g[B.g_off + j] = W[B.w_off + qidx[B.qoff + j]];
}

// W[box][Q_j] = h[box][j]   (W cleared before)
__global__ __launch_bounds__(256) void k_ib_qscatter(const double* __restrict__ hv,
                                                     const BoxDev* __restrict__ boxes,
                                                     const int* __restrict__ qidx,
                                                     double* __restrict__ W) {
  const BoxDev& B = boxes[blockIdx.y];
  for (int j = blockIdx.x * 256 + threadIdx.x; j < B.m; j += gridDim.x * 256)
    W[B.w_off + qidx[B.qoff + j]] = hv[B.g_off + j];
}

__global__ __launch_bounds__(256) void k_ib_fill(double* __restrict__ p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256)
    p[i] = v;
}

// h = C^{-1} g for up to 16 boxes that share C^{-1}.  C^{-1} is symmetric,
// so h_i = sum_k C^{-1}[k][i] g_k streams rows of C^{-1}.  An item (matrix,
// first output i0, first entry in the grouped box list, count) and a k-range
// index (blockIdx.y) own outputs i0 .. i0 + 255 for the item's boxes and
// rows k of one range of kr (a multiple of 64, chosen at setup so that the
// launch has enough workgroups to fill the GPU): every row is read as one
// 2 KB contiguous segment (a thread per output column), 16 rows in flight
// per thread, and the g values of 64 rows at a time sit in LDS.  Partial
// sums per range go to `part` and k_ib_creduce adds the ranges in a fixed
// order.
constexpr int kGC = 256;    // output columns per item
constexpr int kGG = 64;     // g rows staged per step
__global__ __launch_bounds__(256) void k_ib_cgemv(const double* __restrict__ Cinv,
                                                  const IBCorrDev* __restrict__ corr,
                                                  const int4* __restrict__ items,
                                                  const int* __restrict__ gbox,
                                                  const BoxDev* __restrict__ boxes,
                                                  const double* __restrict__ g, int ngbox,
                                                  int m_max, int kr, double* __restrict__ part) {
  __shared__ double gs[kGG][16];
  const int4 it = items[blockIdx.x];
  const IBCorrDev C = corr[it.x];
  const int kb = blockIdx.y * kr;
  if (kb >= C.m) return;                          // this matrix has fewer ranges
  const int ke = min(kb + kr, C.m);
  const int t = threadIdx.x;
  const int i = it.y + t;
  const bool valid = i < C.m;
  const double* M = Cinv + C.off + (valid ? i : 0);
  const int nb = it.w;
  double acc[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) acc[b] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += kGG) {
    const int kc = min(kGG, ke - k0);
    for (int e = t; e < kGG * 16; e += 256) {
      const int kk = e >> 4, b = e & 15;
      gs[kk][b] = (b < nb && kk < kc) ? g[boxes[gbox[it.z + b]].g_off + k0 + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll 16
    for (int kk = 0; kk < kc; ++kk) {
      const double cv = M[(long long)(k0 + kk) * C.mp];
#pragma unroll
      for (int b = 0; b < 16; ++b) acc[b] = __builtin_fma(cv, gs[kk][b], acc[b]);
    }
    __syncthreads();
  }
  if (!valid) return;
  for (int b = 0; b < nb; ++b)
    part[((long long)blockIdx.y * ngbox + it.z + b) * m_max + i] = acc[b];
}

// h[box][i] = sum over the k-ranges of the partial sums, in range order
__global__ __launch_bounds__(256) void k_ib_creduce(const double* __restrict__ part,
                                                    const IBCorrDev* __restrict__ corr,
                                                    const int* __restrict__ gbox,
                                                    const BoxDev* __restrict__ boxes,
                                                    int ngbox, int m_max, int kr,
                                                    double* __restrict__ hv) {
  const int e = blockIdx.y;
  const BoxDev& B = boxes[gbox[e]];
  const int m = B.m;
  const int nr = (m + kr - 1) / kr;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
    double s = 0.0;
    for (int r = 0; r < nr; ++r) s += part[((long long)r * ngbox + e) * m_max + i];
    hv[B.g_off + i] = s;
  }
  (void)corr;
}

// ---------------------------------------------------------------- setup kernels
// unit vectors: Wu[u][Q_{j0+u}] = 1 (Wu cleared before)
__global__ void k_ib_unit(double* __restrict__ Wu, long long stride, const int* __restrict__ q,
                          int nu) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < nu) Wu[(long long)u * stride + q[u]] = 1.0;
}

// C[j0 + u][i] = Wu[u][Q_i] + (i == j0 + u) W^{-1}_i  for i < m (row j0 + u of C;
// A0^{-1} e_j restricted to Q is column j of the symmetric C)
__global__ __launch_bounds__(256) void k_ib_cgather(const double* __restrict__ Wu, long long stride,
                                                    const int* __restrict__ q,
                                                    const double* __restrict__ winv, int m,
                                                    int mp, int j0, double* __restrict__ Cm) {
  const int u = blockIdx.y;
  const int j = j0 + u;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256)
    Cm[(long long)j * mp + i] = Wu[(long long)u * stride + q[i]] + (i == j ? winv[i] : 0.0);
}

// mp x mp identity
__global__ __launch_bounds__(256) void k_ib_ident(double* __restrict__ A, int mp) {
  const long long n = (long long)mp * mp;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n;
       e += (long long)gridDim.x * 256)
    A[e] = (e / mp == e % mp) ? 1.0 : 0.0;
}

// A = (A + A^T) / 2 (each pair i < j handled by one thread)
__global__ __launch_bounds__(256) void k_ib_symm(double* __restrict__ A, int mp) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i < j && j < mp) {
    const double v = 0.5 * (A[(long long)i * mp + j] + A[(long long)j * mp + i]);
    A[(long long)i * mp + j] = v;
    A[(long long)j * mp + i] = v;
  }
}

// Blocked Gauss-Jordan inversion in place, block k (64 rows / columns at k0):
//   P = A_kk^{-1};  Row = P A_k,: ;  Col = A_:,k (copy);
//   A_ij -= Col_i Row_j (i, j != k);  A_kj = Row_j;  A_ik = -Col_i P;  A_kk = P.
constexpr int kGB = 64;
// rank-64 updates of the inversion on the matrix cores (FP64 MFMA) or the vector ALU
constexpr bool kGJMatrixCores = true;

__global__ __launch_bounds__(256) void k_gj_pivot(const double* __restrict__ A, int mp, int k0,
                                                  double* __restrict__ P) {
  __shared__ double a[kGB][kGB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kGB * kGB; e += 256) a[e / kGB][e % kGB] = A[(long long)(k0 + e / kGB) * mp + k0 + e % kGB];
  __syncthreads();
  for (int p = 0; p < kGB; ++p) {
    const double rp = 1.0 / a[p][p];               // one division per thread and step
    double upd[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = t + 256 * r, i = e / kGB, j = e % kGB;
      upd[r] = (i != p && j != p) ? a[i][j] - a[i][p] * (a[p][j] * rp) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = t + 256 * r, i = e / kGB, j = e % kGB;
      if (i != p && j != p) a[i][j] = upd[r];
      else if (i == p && j == p) a[i][j] = rp;
      else if (i == p) a[i][j] = a[i][j] * rp;
      else a[i][j] = -a[i][j] * rp;
    }
    __syncthreads();
  }
  for (int e = t; e < kGB * kGB; e += 256) P[e] = a[e / kGB][e % kGB];
}

// Row[:, J] = P A[k-block rows][J tile];  Col[J tile rows][:] = A[J tile rows][k-block]
__global__ __launch_bounds__(256) void k_gj_panels(const double* __restrict__ A, int mp, int k0,
                                                   const double* __restrict__ P,
                                                   double* __restrict__ Row,
                                                   double* __restrict__ Col) {
  __shared__ double p[kGB][kGB + 1], a[kGB][kGB + 1];
  const int J = blockIdx.x * kGB;
  const int t = threadIdx.x;
  for (int e = t; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    p[i][j] = P[e];
    a[i][j] = A[(long long)(k0 + i) * mp + J + j];
    Col[(long long)(J + i) * kGB + j] = A[(long long)(J + i) * mp + k0 + j];
  }
  __syncthreads();
  const int ti = t >> 4, tj = t & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = ti * 4 + r, j = tj + 16 * c;
      double s = 0.0;
      for (int l = 0; l < kGB; ++l) s = __builtin_fma(p[i][l], a[l][j], s);
      Row[(long long)i * mp + J + j] = s;
    }
}

__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, int mp, int kb,
                                                   const double* __restrict__ P,
                                                   const double* __restrict__ Row,
                                                   const double* __restrict__ Col) {
  __shared__ double cl[kGB][kGB + 1], rw[kGB][kGB + 1];
  const int I = blockIdx.y, J = blockIdx.x;
  const int t = threadIdx.x;
  const long long r0 = (long long)I * kGB, c0 = (long long)J * kGB;
  if (I == kb) {                                  // block row k: Row (or P on the diagonal)
    for (int e = t; e < kGB * kGB; e += 256) {
      const int i = e / kGB, j = e % kGB;
      A[(r0 + i) * mp + c0 + j] = (J == kb) ? P[e] : Row[(long long)i * mp + c0 + j];
    }
    return;
  }
  for (int e = t; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    cl[i][j] = Col[(r0 + i) * kGB + j];
    rw[i][j] = (J == kb) ? P[e] : Row[(long long)i * mp + c0 + j];
  }
  __syncthreads();
  const int ti = t >> 4, tj = t & 15;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
#pragma unroll 4
  for (int l = 0; l < kGB; ++l) {
    double av[4], bv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = cl[ti * 4 + r][l];
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[c] = rw[l][tj + 16 * c];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_fma(av[r], bv[c], acc[r][c]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long idx = (r0 + ti * 4 + r) * mp + c0 + tj + 16 * c;
      A[idx] = (J == kb) ? -acc[r][c] : A[idx] - acc[r][c];
    }
}

// The same update on the matrix cores: v_mfma_f64_16x16x4f64 with lane l
// holding A[l % 16][l / 16] and B[l / 16][l % 16] and the accumulator's
// element i at D[4 i + l / 16][l % 16] (measured on gfx950).  Wave w computes rows 16 w .. + 15
// of the 64 x 64 tile against its four 16-column tiles, 16 k-steps of 4.
typedef double d4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_gj_update_mfma(double* __restrict__ A, int mp, int kb,
                                                        const double* __restrict__ P,
                                                        const double* __restrict__ Row,
                                                        const double* __restrict__ Col) {
  __shared__ double cl[kGB][kGB + 1], rw[kGB][kGB + 1];
  const int I = blockIdx.y, J = blockIdx.x;
  const int t = threadIdx.x;
  const long long r0 = (long long)I * kGB, c0 = (long long)J * kGB;
  if (I == kb) {                                  // block row k: Row (or P on the diagonal)
    for (int e = t; e < kGB * kGB; e += 256) {
      const int i = e / kGB, j = e % kGB;
      A[(r0 + i) * mp + c0 + j] = (J == kb) ? P[e] : Row[(long long)i * mp + c0 + j];
    }
    return;
  }
  for (int e = t; e < kGB * kGB; e += 256) {
    const int i = e / kGB, j = e % kGB;
    cl[i][j] = Col[(r0 + i) * kGB + j];
    rw[i][j] = (J == kb) ? P[e] : Row[(long long)i * mp + c0 + j];
  }
  __syncthreads();
  const int w = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
  d4_t acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = d4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int ks = 0; ks < kGB / 4; ++ks) {
    const double a = cl[16 * w + lr][4 * ks + lk];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      acc[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rw[4 * ks + lk][16 * nt + lr], acc[nt], 0, 0, 0);
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long idx = (r0 + 16 * w + 4 * i + lk) * mp + c0 + 16 * nt + lr;
      A[idx] = (J == kb) ? -acc[nt][i] : A[idx] - acc[nt][i];
    }
}

int blocks_for(long long n) { return (int)std::min<long long>((n + 255) / 256, 4096); }

#define FMP_IB_SWITCH(NP, CALL)            \
  switch (NP) {                            \
    case 8: return CALL(8);                \
    case 16: return CALL(16);              \
    case 24: return CALL(24);              \
    case 32: return CALL(32);              \
    case 34: return CALL(34);              \
    case 48: return CALL(48);              \
    default: return hipErrorInvalidValue;  \
  }

template <int NP>
hipError_t run_ib_a(const double* r, const double* Win, double* W, const BoxDev* boxes,
                    const DomainDev* doms, const int4* work, int nwork, const double* tab,
                    hipStream_t s) {
  hipLaunchKernelGGL((k_ib_a<NP>), dim3(nwork), dim3(kIBT), 0, s, r, Win, W, boxes, doms, work, tab);
  return hipGetLastError();
}
template <int NP>
hipError_t run_ib_b(double* W, const BoxDev* boxes, const int4* work, int nwork,
                    const double* tab, hipStream_t s) {
  hipLaunchKernelGGL((k_ib_b<NP>), dim3(nwork), dim3(192), 0, s, W, boxes, work, tab);
  return hipGetLastError();
}
template <int NP>
hipError_t run_ib_c(const double* Wsrc, double* Wdst, const double* E, double* z,
                    const BoxDev* boxes, const DomainDev* doms, const int4* work, int nwork,
                    const double* tab, hipStream_t s) {
  hipLaunchKernelGGL((k_ib_c<NP>), dim3(nwork), dim3(kIBT), 0, s, Wsrc, Wdst, E, z, boxes, doms,
                     work, tab);
  return hipGetLastError();
}

}  // namespace

int ib_class_np(int cls) { return kIBClasses[cls]; }
int ib_class_of(int n) {
  for (int c = 0; c < kNumIBClasses; ++c)
    if (kIBClasses[c] >= n) return c;
  return -1;
}
int ib_zslab(int np) { return kIBT / np > 0 ? kIBT / np : 1; }

hipError_t launch_ib_a(int np, const double* r, const double* Win, double* W, const BoxDev* boxes,
                       const DomainDev* doms, const int4* work, int nwork, const double* tab,
                       hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
#define CALL(N) run_ib_a<N>(r, Win, W, boxes, doms, work, nwork, tab, s)
  FMP_IB_SWITCH(np, CALL)
#undef CALL
}
hipError_t launch_ib_b(int np, double* W, const BoxDev* boxes, const int4* work, int nwork,
                       const double* tab, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
#define CALL(N) run_ib_b<N>(W, boxes, work, nwork, tab, s)
  FMP_IB_SWITCH(np, CALL)
#undef CALL
}
hipError_t launch_ib_c(int np, const double* Wsrc, double* Wdst, const double* E, double* z,
                       const BoxDev* boxes, const DomainDev* doms, const int4* work, int nwork,
                       const double* tab, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
#define CALL(N) run_ib_c<N>(Wsrc, Wdst, E, z, boxes, doms, work, nwork, tab, s)
  FMP_IB_SWITCH(np, CALL)
#undef CALL
}

}  // namespace fmp

using namespace fmp;

namespace {

constexpr size_t kAl = 256;
size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }

// Closed-form compact-difference bases of side n into the table slot at base.
void compact_tables(int n, double* base) {
  double* Uf = base;                              // U^T: rows m, columns i
  double* Ui = base + kIT * kIT;                  // U:   rows i, columns m
  double* Vf = base + 2 * kIT * kIT;
  double* Vi = base + 3 * kIT * kIT;
  double* sg = base + 4 * kIT * kIT;
  const double c = 2.0 / sqrt(2.0 * n + 1.0);
  for (int m = 0; m < n; ++m) {
    const double th = (2.0 * m + 1.0) * M_PI / (2.0 * n + 1.0);   // theta_{m+1}
    sg[m] = 2.0 * sin(0.5 * th);
    for (int i = 0; i < n; ++i) {
      const double u = -c * sin(th * (i + 1.0));
      const double v = c * cos(th * (i + 0.5));
      Uf[m * kIT + i] = u;
      Ui[i * kIT + m] = u;
      Vf[m * kIT + i] = v;
      Vi[i * kIT + m] = v;
    }
  }
}

// Q of a box shape: flattened (q, z, y, x) slots on a low face of a node axis,
// in that order; delta and the wall flag of each slot.
void boundary_slots(int nx, int ny, int nz, int wall, std::vector<int>* idx,
                    std::vector<int>* delta, std::vector<char>* is_wall) {
  const int L[3] = {nx, ny, nz};
  const long long vol = (long long)nx * ny * nz;
  for (int q = 0; q < 3; ++q)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int pos[3] = {x, y, z};
          int d = 0;
          bool w = false;
          for (int a = 0; a < 3; ++a) {
            if (a == q || pos[a] != 0) continue;
            ++d;
            if ((wall >> a) & 1) w = true;
          }
          (void)L;
          if (d == 0) continue;
          if (idx) idx->push_back((int)(q * vol + ((long long)z * ny + y) * nx + x));
          if (delta) delta->push_back(d);
          if (is_wall) is_wall->push_back(w ? 1 : 0);
        }
}

void add_work(const BoxDev& B, int bi, int np, std::vector<int4>* wa, std::vector<int4>* wb) {
  const int zs = ib_zslab(np);
  for (int q = 0; q < 3; ++q)
    for (int z0 = 0; z0 < B.nz; z0 += zs) wa->push_back(make_int4(bi, q, z0, 0));
  for (int c0 = 0; c0 < B.nx * B.ny; c0 += 64) wb->push_back(make_int4(bi, c0, 0, 0));
}

fmp_status hipfail(fmp_ctx* h, hipError_t e, const char* what) {
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  return FMP_ERR_HIP;
}

#define IBCHK(call)                                   \
  do {                                                \
    const hipError_t _e = (call);                     \
    if (_e != hipSuccess) return hipfail(h, _e, #call); \
  } while (0)

}  // namespace

// Plans of the index-block path.  The generic setup has put the boxes (index
// ranges of owned block plus overlap, clipped at the grid, and alpha) into
// h->boxes; they move to h->ib.
fmp_status ib_prepare(fmp_ctx* h) {
  IBPlan& P = h->ib;
  P.on = true;
  P.boxes.swap(h->boxes);
  h->boxes.clear();
  // tables per distinct side
  std::vector<int> slot(kIBMaxSide + 1, -1);
  int nsides = 0;
  for (const BoxDev& B : P.boxes)
    for (int n : {B.nx, B.ny, B.nz}) {
      if (n < 1 || n > kIBMaxSide) {
        h->err = "index-block boxes are limited to sides of 1.." + std::to_string(kIBMaxSide);
        return FMP_ERR_UNSUPPORTED;
      }
      if (slot[n] < 0) slot[n] = nsides++;
    }
  P.tab.assign((size_t)(kIBPerSide * nsides), 0.0);
  for (int n = 1; n <= kIBMaxSide; ++n)
    if (slot[n] >= 0) compact_tables(n, P.tab.data() + slot[n] * kIBPerSide);
  // boundary slot lists per shape, corrections per (shape, walls, alpha)
  std::map<std::tuple<int, int, int>, int> shape_q;
  std::map<std::tuple<int, int, int, int, double>, int> corr_of;
  long long g = 0, vmax = 0;
  for (size_t bi = 0; bi < P.boxes.size(); ++bi) {
    BoxDev& B = P.boxes[bi];
    const int sides[3] = {B.nx, B.ny, B.nz};
    for (int a = 0; a < 3; ++a) B.ibt[a] = (int)(slot[sides[a]] * kIBPerSide);
    B.wall = (B.bx0 == 0 ? 1 : 0) | (B.by0 == 0 ? 2 : 0) | (B.bz0 == 0 ? 4 : 0);
    const auto sk = std::make_tuple(B.nx, B.ny, B.nz);
    auto it = shape_q.find(sk);
    if (it == shape_q.end()) {
      const int off = (int)P.qidx.size();
      boundary_slots(B.nx, B.ny, B.nz, 0, &P.qidx, nullptr, nullptr);
      it = shape_q.emplace(sk, off).first;
    }
    B.qoff = it->second;
    B.m = (int)((long long)B.nx * B.ny * B.nz * 3 - (long long)B.nx * (B.ny - 1) * (B.nz - 1) -
                (long long)(B.nx - 1) * B.ny * (B.nz - 1) - (long long)(B.nx - 1) * (B.ny - 1) * B.nz);
    if (!(B.alpha > 0.0)) B.m = 0;               // A = I: no boundary correction
    const auto ck = std::make_tuple(B.nx, B.ny, B.nz, B.wall, B.alpha);
    auto ci = corr_of.find(ck);
    if (B.m > 0 && ci == corr_of.end()) {
      IBCorr C{};
      C.nx = B.nx; C.ny = B.ny; C.nz = B.nz; C.wall = B.wall; C.alpha = B.alpha;
      C.m = B.m;
      C.mp = (B.m + kGB - 1) / kGB * kGB;
      C.qoff = B.qoff;
      C.off = P.cinv_elems;
      C.rep = (int)bi;
      P.cinv_elems += (long long)C.mp * C.mp;
      P.m_max = std::max(P.m_max, C.m);
      P.mp_max = std::max(P.mp_max, C.mp);
      ci = corr_of.emplace(ck, (int)P.corr.size()).first;
      P.corr.push_back(C);
    }
    B.corr = B.m > 0 ? ci->second : -1;
    B.g_off = g;
    g += (B.m + 7) / 8 * 8;
    B.w_off = P.w_elems;
    P.w_elems += (3 * B.vol + 7) / 8 * 8;
    vmax = std::max(vmax, B.vol);
  }
  P.g_elems = std::max<long long>(g, 8);
  P.vol_max = vmax;
  // classes and work lists (boxes in class order)
  for (int c = 0; c < kNumIBClasses; ++c) {
    IBPlan::Cls cl{kIBClasses[c], (int)P.work_a.size(), 0, (int)P.work_b.size(), 0};
    for (size_t bi = 0; bi < P.boxes.size(); ++bi) {
      const BoxDev& B = P.boxes[bi];
      if (ib_class_of(std::max(B.nx, std::max(B.ny, B.nz))) != c) continue;
      add_work(B, (int)bi, cl.np, &P.work_a, &P.work_b);
    }
    cl.na = (int)P.work_a.size() - cl.a0;
    cl.nb = (int)P.work_b.size() - cl.b0;
    if (cl.na) P.cls.push_back(cl);
  }
  // C^{-1} h items: boxes grouped by matrix, 16 at a time, kGC outputs per item
  for (size_t k = 0; k < P.corr.size(); ++k) {
    const int first = (int)P.gbox.size();
    for (size_t bi = 0; bi < P.boxes.size(); ++bi)
      if (P.boxes[bi].corr == (int)k) P.gbox.push_back((int)bi);
    const int cnt = (int)P.gbox.size() - first;
    for (int b0 = 0; b0 < cnt; b0 += 16)
      for (int i0 = 0; i0 < P.corr[k].m; i0 += kGC)
        P.gemv.push_back(make_int4((int)k, i0, first + b0, std::min(16, cnt - b0)));
  }
  // k-range: the longest (fewest partial sums) that still gives the launch
  // about 2048 workgroups (8 per CU)
  P.gemv_kr = 1024;
  while (P.gemv_kr > 256 &&
         (long long)P.gemv.size() * ((P.m_max + P.gemv_kr - 1) / P.gemv_kr) < 2048)
    P.gemv_kr /= 2;
  // setup batches of unit solves reuse the W_E + W_C region
  P.unit_batch = std::max(1, std::min(P.m_max, 128));
  P.stage_elems = std::max(2 * P.w_elems, (long long)P.unit_batch * ((3 * vmax + 7) / 8 * 8));
  return FMP_OK;
}

// partial sums of the C^{-1} h step: k-ranges x grouped boxes x m_max
static size_t gemv_part_elems(const IBPlan& P) {
  const size_t nr = (size_t)(P.m_max + P.gemv_kr - 1) / P.gemv_kr;
  return nr * P.gbox.size() * (size_t)P.m_max;
}

size_t ib_workspace_bytes(const fmp_ctx* h) {
  const IBPlan& P = h->ib;
  size_t b = 0;
  b += al(std::max<size_t>(P.boxes.size(), 1) * sizeof(BoxDev));
  b += al(std::max<size_t>(P.tab.size(), 1) * 8);
  b += al(std::max<size_t>(P.qidx.size(), 1) * 4);
  b += al(std::max<size_t>(P.corr.size(), 1) * sizeof(IBCorrDev));
  b += al(std::max<size_t>(P.work_a.size(), 1) * sizeof(int4));
  b += al(std::max<size_t>(P.work_b.size(), 1) * sizeof(int4));
  b += al(std::max<size_t>(P.gemv.size(), 1) * sizeof(int4));
  b += al(std::max<size_t>(P.gbox.size(), 1) * 4);
  b += al((size_t)P.stage_elems * 8);
  b += 2 * al((size_t)P.g_elems * 8);
  b += al(std::max<size_t>(gemv_part_elems(P), 1) * 8);
  b += al(std::max<long long>(P.cinv_elems, 1) * 8);
  // setup only
  b += al((size_t)kGB * kGB * 8);
  b += 2 * al((size_t)std::max(P.mp_max, kGB) * kGB * 8);
  b += al((size_t)std::max(P.m_max, 1) * 8);
  b += al((size_t)P.unit_batch * sizeof(BoxDev));
  const int np_max = 48;
  const long long ua = (long long)P.unit_batch * 3 * ((kIBMaxSide + ib_zslab(8) - 1));
  (void)np_max;
  b += al((size_t)std::max<long long>(ua, 1) * sizeof(int4));
  b += al((size_t)P.unit_batch * ((kIBMaxSide * kIBMaxSide + 63) / 64) * sizeof(int4));
  return b;
}

fmp_status ib_bind(fmp_ctx* h, char* base, hipStream_t s) {
  IBPlan& P = h->ib;
  char* p = base;
  auto take = [&](size_t bytes) { char* r = p; p += al(bytes); return r; };
  P.d_boxes = (BoxDev*)take(std::max<size_t>(P.boxes.size(), 1) * sizeof(BoxDev));
  P.d_tab = (double*)take(std::max<size_t>(P.tab.size(), 1) * 8);
  P.d_qidx = (int*)take(std::max<size_t>(P.qidx.size(), 1) * 4);
  P.d_corr = (IBCorrDev*)take(std::max<size_t>(P.corr.size(), 1) * sizeof(IBCorrDev));
  P.d_work_a = (int4*)take(std::max<size_t>(P.work_a.size(), 1) * sizeof(int4));
  P.d_work_b = (int4*)take(std::max<size_t>(P.work_b.size(), 1) * sizeof(int4));
  P.d_gemv = (int4*)take(std::max<size_t>(P.gemv.size(), 1) * sizeof(int4));
  P.d_gbox = (int*)take(std::max<size_t>(P.gbox.size(), 1) * 4);
  double* stage = (double*)take((size_t)P.stage_elems * 8);
  P.d_WE = stage;
  P.d_WC = stage + P.w_elems;
  P.d_g = (double*)take((size_t)P.g_elems * 8);
  P.d_hv = (double*)take((size_t)P.g_elems * 8);
  P.d_part = (double*)take(std::max<size_t>(gemv_part_elems(P), 1) * 8);
  P.d_cinv = (double*)take(std::max<long long>(P.cinv_elems, 1) * 8);
  P.d_P = (double*)take((size_t)kGB * kGB * 8);
  P.d_Row = (double*)take((size_t)std::max(P.mp_max, kGB) * kGB * 8);
  P.d_Col = (double*)take((size_t)std::max(P.mp_max, kGB) * kGB * 8);
  P.d_winv = (double*)take((size_t)std::max(P.m_max, 1) * 8);
  P.d_ubox = (BoxDev*)take((size_t)P.unit_batch * sizeof(BoxDev));
  const long long ua = (long long)P.unit_batch * 3 * ((kIBMaxSide + ib_zslab(8) - 1));
  P.d_uwork_a = (int4*)take((size_t)std::max<long long>(ua, 1) * sizeof(int4));
  P.d_uwork_b = (int4*)take((size_t)P.unit_batch * ((kIBMaxSide * kIBMaxSide + 63) / 64) * sizeof(int4));
  if ((size_t)(p - base) > ib_workspace_bytes(h)) {
    h->err = "index-block workspace layout";
    return FMP_ERR_WORKSPACE;
  }

  std::vector<IBCorrDev> cd(P.corr.size());
  for (size_t k = 0; k < P.corr.size(); ++k) cd[k] = IBCorrDev{P.corr[k].off, P.corr[k].m, P.corr[k].mp};
  IBCHK(hipMemcpyAsync(P.d_boxes, P.boxes.data(), P.boxes.size() * sizeof(BoxDev), hipMemcpyHostToDevice, s));
  IBCHK(hipMemcpyAsync(P.d_tab, P.tab.data(), P.tab.size() * 8, hipMemcpyHostToDevice, s));
  if (!P.qidx.empty())
    IBCHK(hipMemcpyAsync(P.d_qidx, P.qidx.data(), P.qidx.size() * 4, hipMemcpyHostToDevice, s));
  if (!cd.empty())
    IBCHK(hipMemcpyAsync(P.d_corr, cd.data(), cd.size() * sizeof(IBCorrDev), hipMemcpyHostToDevice, s));
  IBCHK(hipMemcpyAsync(P.d_work_a, P.work_a.data(), P.work_a.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  IBCHK(hipMemcpyAsync(P.d_work_b, P.work_b.data(), P.work_b.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  if (!P.gemv.empty()) {
    IBCHK(hipMemcpyAsync(P.d_gemv, P.gemv.data(), P.gemv.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    IBCHK(hipMemcpyAsync(P.d_gbox, P.gbox.data(), P.gbox.size() * 4, hipMemcpyHostToDevice, s));
  }
  IBCHK(hipStreamSynchronize(s));

  // ---- C^{-1} for every correction: unit solves, C, symmetric, invert
  const int U = P.unit_batch;
  for (size_t k = 0; k < P.corr.size(); ++k) {
    const IBCorr& C = P.corr[k];
    const BoxDev& R = P.boxes[C.rep];
    std::vector<int> qi, dl;
    std::vector<char> wl;
    boundary_slots(C.nx, C.ny, C.nz, C.wall, &qi, &dl, &wl);
    if ((int)qi.size() != C.m) {
      h->err = "index-block boundary slot count";
      return FMP_ERR_UNSUPPORTED;
    }
    std::vector<double> winv(C.m);
    for (int j = 0; j < C.m; ++j) winv[j] = wl[j] ? 0.0 : 1.0 / (C.alpha * dl[j]);
    const long long stride = (3 * R.vol + 7) / 8 * 8;
    std::vector<BoxDev> ub(U, R);
    for (int u = 0; u < U; ++u) ub[u].w_off = (long long)u * stride;
    const int np = ib_class_np(ib_class_of(std::max(R.nx, std::max(R.ny, R.nz))));
    std::vector<int4> ua, ubw;
    for (int u = 0; u < U; ++u) add_work(ub[u], u, np, &ua, &ubw);
    const int na_per = (int)ua.size() / U, nb_per = (int)ubw.size() / U;
    IBCHK(hipMemcpyAsync(P.d_winv, winv.data(), C.m * 8, hipMemcpyHostToDevice, s));
    IBCHK(hipMemcpyAsync(P.d_ubox, ub.data(), U * sizeof(BoxDev), hipMemcpyHostToDevice, s));
    IBCHK(hipMemcpyAsync(P.d_uwork_a, ua.data(), ua.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    IBCHK(hipMemcpyAsync(P.d_uwork_b, ubw.data(), ubw.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    double* Cm = P.d_cinv + C.off;
    hipLaunchKernelGGL(k_ib_ident, dim3(blocks_for((long long)C.mp * C.mp)), dim3(256), 0, s, Cm, C.mp);
    IBCHK(hipGetLastError());
    const int* q = P.d_qidx + C.qoff;
    double* Wu = P.d_WE;
    for (int j0 = 0; j0 < C.m; j0 += U) {
      const int nu = std::min(U, C.m - j0);
      hipLaunchKernelGGL(k_ib_fill, dim3(blocks_for(nu * stride)), dim3(256), 0, s, Wu,
                         (long long)nu * stride, 0.0);
      hipLaunchKernelGGL(k_ib_unit, dim3((nu + 63) / 64), dim3(64), 0, s, Wu, stride, q + j0, nu);
      IBCHK(hipGetLastError());
      IBCHK(launch_ib_a(np, nullptr, Wu, Wu, P.d_ubox, h->d_doms, P.d_uwork_a, nu * na_per,
                        P.d_tab, s));
      IBCHK(launch_ib_b(np, Wu, P.d_ubox, P.d_uwork_b, nu * nb_per, P.d_tab, s));
      IBCHK(launch_ib_c(np, Wu, Wu, nullptr, nullptr, P.d_ubox, h->d_doms, P.d_uwork_a,
                        nu * na_per, P.d_tab, s));
      hipLaunchKernelGGL(k_ib_cgather, dim3((C.m + 255) / 256, nu), dim3(256), 0, s, Wu, stride,
                         q, P.d_winv, C.m, C.mp, j0, Cm);
      IBCHK(hipGetLastError());
    }
    const dim3 sg((C.mp + 15) / 16, (C.mp + 15) / 16);
    hipLaunchKernelGGL(k_ib_symm, sg, dim3(256), 0, s, Cm, C.mp);
    const int nblk = C.mp / kGB;
    for (int kb = 0; kb < nblk; ++kb) {
      hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, Cm, C.mp, kb * kGB, P.d_P);
      hipLaunchKernelGGL(k_gj_panels, dim3(nblk), dim3(256), 0, s, Cm, C.mp, kb * kGB, P.d_P,
                         P.d_Row, P.d_Col);
      if (kGJMatrixCores)
        hipLaunchKernelGGL(k_gj_update_mfma, dim3(nblk, nblk), dim3(256), 0, s, Cm, C.mp, kb,
                           P.d_P, P.d_Row, P.d_Col);
      else
        hipLaunchKernelGGL(k_gj_update, dim3(nblk, nblk), dim3(256), 0, s, Cm, C.mp, kb, P.d_P,
                           P.d_Row, P.d_Col);
    }
    hipLaunchKernelGGL(k_ib_symm, sg, dim3(256), 0, s, Cm, C.mp);
    IBCHK(hipGetLastError());
    IBCHK(hipStreamSynchronize(s));               // host staging of this matrix goes out of scope
  }
  return FMP_OK;
}

fmp_status ib_apply(fmp_ctx* h, const double* r, double* z, hipStream_t s) {
  IBPlan& P = h->ib;
  // E = exact_solve(S^gamma r) in W_E
  for (const auto& c : P.cls)
    IBCHK(launch_ib_a(c.np, r, nullptr, P.d_WE, P.d_boxes, h->d_doms, P.d_work_a + c.a0, c.na, P.d_tab, s));
  for (const auto& c : P.cls)
    IBCHK(launch_ib_b(c.np, P.d_WE, P.d_boxes, P.d_work_b + c.b0, c.nb, P.d_tab, s));
  const int nbox = (int)P.boxes.size();
  if (P.corr.empty()) {                           // no boundary correction (alpha = 0)
    for (const auto& c : P.cls)
      IBCHK(launch_ib_c(c.np, P.d_WE, nullptr, nullptr, nullptr, P.d_boxes, h->d_doms,
                        P.d_work_a + c.a0, c.na, P.d_tab, s));
    // z = E on the owned unknowns: pass C with W_C = 0 subtracted
    hipLaunchKernelGGL(k_ib_fill, dim3(blocks_for(P.w_elems)), dim3(256), 0, s, P.d_WC, P.w_elems, 0.0);
    IBCHK(hipGetLastError());
  } else {
    for (const auto& c : P.cls)
      IBCHK(launch_ib_c(c.np, P.d_WE, P.d_WE, nullptr, nullptr, P.d_boxes, h->d_doms,
                        P.d_work_a + c.a0, c.na, P.d_tab, s));
    // g = Q^T E, h = C^{-1} g, W_C = Q h
    const int mblk = std::max(1, std::min(64, (P.m_max + 255) / 256));
    hipLaunchKernelGGL(k_ib_qgather, dim3(mblk, nbox), dim3(256), 0, s, P.d_WE, P.d_boxes, P.d_qidx, P.d_g);
    const int kr = P.gemv_kr, nr = (P.m_max + kr - 1) / kr, ngb = (int)P.gbox.size();
    hipLaunchKernelGGL(k_ib_cgemv, dim3((int)P.gemv.size(), nr), dim3(256), 0, s, P.d_cinv,
                       P.d_corr, P.d_gemv, P.d_gbox, P.d_boxes, P.d_g, ngb, P.m_max, kr, P.d_part);
    hipLaunchKernelGGL(k_ib_creduce, dim3(std::min(64, (P.m_max + 255) / 256), ngb), dim3(256), 0,
                       s, P.d_part, P.d_corr, P.d_gbox, P.d_boxes, ngb, P.m_max, kr, P.d_hv);
    hipLaunchKernelGGL(k_ib_fill, dim3(blocks_for(P.w_elems)), dim3(256), 0, s, P.d_WC, P.w_elems, 0.0);
    hipLaunchKernelGGL(k_ib_qscatter, dim3(mblk, nbox), dim3(256), 0, s, P.d_hv, P.d_boxes, P.d_qidx, P.d_WC);
    IBCHK(hipGetLastError());
    // CorE = exact_solve(W_C) (passes A, B in place)
    for (const auto& c : P.cls)
      IBCHK(launch_ib_a(c.np, nullptr, P.d_WC, P.d_WC, P.d_boxes, h->d_doms, P.d_work_a + c.a0, c.na, P.d_tab, s));
    for (const auto& c : P.cls)
      IBCHK(launch_ib_b(c.np, P.d_WC, P.d_boxes, P.d_work_b + c.b0, c.nb, P.d_tab, s));
  }
  // z = S^0T (E - CorE): pass C of W_C, subtracted from W_E on the owned unknowns
  for (const auto& c : P.cls)
    IBCHK(launch_ib_c(c.np, P.d_WC, nullptr, P.d_WE, z, P.d_boxes, h->d_doms, P.d_work_a + c.a0,
                      c.na, P.d_tab, s));
  return FMP_OK;
}
