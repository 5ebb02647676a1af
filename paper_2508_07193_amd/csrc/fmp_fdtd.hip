// Crank-Nicolson time stepping around the solve (Sec. II-A, eqs. (2)-(5)).
//
// With mu = 1 and unit cell size, eq. (3) gives H+ = H - (dt/2) C (E+ + E)
// and eliminating H+ from eq. (2) gives A E+ = R with A = I + c eps^-1 C^T C,
// c = dt^2 / 4 (the operator of the stencil kernel) and
//     R = E + dt eps^-1 C^T (H - (dt/4) C E).
// C is the Yee curl from E (edges) to H (dual faces) of Sec. III-A eq. (6),
// C^T the curl from H back to the edges.  Each domain's dt is 2 sqrt(c).
//
// Two elementwise kernels, one thread per cell (x fastest, all three
// components): the face kernel k_curl_e (h_out = beta h_in + s C (e1 + e2))
// and the edge kernel k_curl_h (e_out = e_in + s eps_e^-1 C^T h), eps_e the
// mean of the four cells sharing the edge, summed in the stencil kernel's
// order.  Both are HBM-bound (8 B in per input vector and 8 B out per slot;
// neighbour reads hit the caches).
#include <cmath>

#include "fmp_ctx.h"

namespace fmp {
namespace {

constexpr int kFX = 64, kFY = 4;

// E slots that are unknowns (slot 0 of a component's two node axes is a wall)
__device__ __forceinline__ bool e_slot(int q, int i, int j, int k) {
  return q == 0 ? (j > 0 && k > 0) : (q == 1 ? (i > 0 && k > 0) : (i > 0 && j > 0));
}
// H slots that are unknowns (slot 0 of the component's own node axis is a wall)
__device__ __forceinline__ bool h_slot(int q, int i, int j, int k) {
  return q == 0 ? i > 0 : (q == 1 ? j > 0 : k > 0);
}

// h_out = beta h_in + s C (e1 + e2):
//   H_x = d_y E_z - d_z E_y,  H_y = d_z E_x - d_x E_z,  H_z = d_x E_y - d_y E_x
// with forward differences to the half points; E beyond the far wall and on
// wall slots is zero.
__global__ __launch_bounds__(kFX * kFY) void k_curl_e(const double* __restrict__ e1,
                                                      const double* __restrict__ e2,
                                                      const double* h_in, double beta, double s,
                                                      double* h_out, DomainDev D) {
  const int i = blockIdx.x * kFX + threadIdx.x, j = blockIdx.y * kFY + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = D.nx, ny = D.ny, nz = D.nz;
  if (i >= nx || j >= ny) return;
  const long long cs = (long long)nz * ny * nx;
  auto E = [&](int q, int kk, int jj, int ii) -> double {
    if (ii >= nx || jj >= ny || kk >= nz || !e_slot(q, ii, jj, kk)) return 0.0;
    const long long o = D.offset + q * cs + ((long long)kk * ny + jj) * nx + ii;
    double v = e1[o];
    if (e2) v += e2[o];
    return v;
  };
  const double ex = E(0, k, j, i), ey = E(1, k, j, i), ez = E(2, k, j, i);
  const double cx = (E(2, k, j + 1, i) - ez) - (E(1, k + 1, j, i) - ey);
  const double cy = (E(0, k + 1, j, i) - ex) - (E(2, k, j, i + 1) - ez);
  const double cz = (E(1, k, j, i + 1) - ey) - (E(0, k, j + 1, i) - ex);
  const long long o = D.offset + ((long long)k * ny + j) * nx + i;
  const double cv[3] = {cx, cy, cz};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double v = 0.0;
    if (h_slot(q, i, j, k)) {
      v = s * cv[q];
      if (h_in) v = beta * h_in[o + q * cs] + v;
    }
    h_out[o + q * cs] = v;
  }
}

// e_out = e_in + s eps_e^-1 C^T h:
//   (C^T H)_x = d_y H_z - d_z H_y,  (C^T H)_y = d_z H_x - d_x H_z,
//   (C^T H)_z = d_x H_y - d_y H_x
// with backward differences from the half points; H on wall slots is zero.
__global__ __launch_bounds__(kFX * kFY) void k_curl_h(const double* __restrict__ hf,
                                                      const double* e_in, double s, double* e_out,
                                                      DomainDev D, const double* __restrict__ eps) {
  const int i = blockIdx.x * kFX + threadIdx.x, j = blockIdx.y * kFY + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = D.nx, ny = D.ny, nz = D.nz;
  if (i >= nx || j >= ny) return;
  const long long cs = (long long)nz * ny * nx;
  auto H = [&](int q, int kk, int jj, int ii) -> double {
    if (ii < 0 || jj < 0 || kk < 0 || !h_slot(q, ii, jj, kk)) return 0.0;
    return hf[D.offset + q * cs + ((long long)kk * ny + jj) * nx + ii];
  };
  const double hx = H(0, k, j, i), hy = H(1, k, j, i), hz = H(2, k, j, i);
  const double cx = (hz - H(2, k, j - 1, i)) - (hy - H(1, k - 1, j, i));
  const double cy = (hx - H(0, k - 1, j, i)) - (hz - H(2, k, j, i - 1));
  const double cz = (hy - H(1, k, j, i - 1)) - (hx - H(0, k, j - 1, i));
  // cells c[dk][dj][di] at (k-1+dk, j-1+dj, i-1+di) (c000 is not needed), clamped
  // into the domain (only wall slots reach outside); eps cube indices from an
  // exact float quotient (v < 2^22)
  double c001 = 1.0, c010 = 1.0, c011 = 1.0, c100 = 1.0, c101 = 1.0, c110 = 1.0, c111 = 1.0;
  if (D.eps_b > 0) {
    const float inv_b = 1.f / (float)D.eps_b;
    auto blk = [&](int v, int n) { return (int)(((float)min(max(v, 0), n - 1) + 0.5f) * inv_b); };
    const int kb0 = blk(k - 1, nz), kb1 = blk(k, nz);
    const int jb0 = blk(j - 1, ny), jb1 = blk(j, ny);
    const int ib0 = blk(i - 1, nx), ib1 = blk(i, nx);
    const double* et = eps + D.eps_off;
    auto at = [&](int kb, int jb, int ib) { return et[((long long)kb * D.eps_nby + jb) * D.eps_nbx + ib]; };
    c001 = at(kb0, jb0, ib1);
    c010 = at(kb0, jb1, ib0);
    c011 = at(kb0, jb1, ib1);
    c100 = at(kb1, jb0, ib0);
    c101 = at(kb1, jb0, ib1);
    c110 = at(kb1, jb1, ib0);
    c111 = at(kb1, jb1, ib1);
  }
  // edge permittivity: mean of the four cells sharing the edge, in the order
  // (-,-), (+,-), (-,+), (+,+) of the two transverse axes
  const double ex_e = 0.25 * (((c001 + c101) + c011) + c111);
  const double ey_e = 0.25 * (((c010 + c110) + c011) + c111);
  const double ez_e = 0.25 * (((c100 + c110) + c101) + c111);
  const long long o = D.offset + ((long long)k * ny + j) * nx + i;
  const double cv[3] = {cx, cy, cz}, ev[3] = {ex_e, ey_e, ez_e};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double v = 0.0;
    if (e_slot(q, i, j, k)) {
      v = (s / ev[q]) * cv[q];
      if (e_in) v = e_in[o + q * cs] + v;
    }
    e_out[o + q * cs] = v;
  }
}

bool overlap_bytes(const void* a, const void* b, long long bytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bytes && pb < pa + bytes;
}

fmp_status hip_status(fmp_ctx* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return FMP_OK;
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  return FMP_ERR_HIP;
}

constexpr size_t kAlignCN = 256;
size_t align_cn(size_t x) { return (x + kAlignCN - 1) / kAlignCN * kAlignCN; }

dim3 cell_grid(const DomainDev& D) {
  return dim3((D.nx + kFX - 1) / kFX, (D.ny + kFY - 1) / kFY, D.nz);
}

}  // namespace
}  // namespace fmp

using fmp::DomainDev;

extern "C" {

fmp_status fmp_curl_e(fmp_handle h, const double* e1, const double* e2, const double* h_in,
                      double beta, double m, double* h_out, void* stream) {
  if (!h || !e1 || !h_out) return FMP_ERR_INVALID_ARG;
  const long long bytes = h->len * 8;
  if (fmp::overlap_bytes(e1, h_out, bytes) || (e2 && fmp::overlap_bytes(e2, h_out, bytes)))
    return FMP_ERR_ALIAS;
  if (h_in && h_in != h_out && fmp::overlap_bytes(h_in, h_out, bytes)) return FMP_ERR_ALIAS;
  hipStream_t s = (hipStream_t)stream;
  for (const DomainDev& D : h->doms) {
    const double sc = m * 2.0 * std::sqrt(D.c);
    hipLaunchKernelGGL(fmp::k_curl_e, fmp::cell_grid(D), dim3(fmp::kFX, fmp::kFY), 0, s, e1, e2,
                       h_in, beta, sc, h_out, D);
    if (fmp_status st = fmp::hip_status(h, hipGetLastError(), "k_curl_e")) return st;
  }
  return FMP_OK;
}

fmp_status fmp_curl_h(fmp_handle h, const double* hf, const double* e_in, double m, double* e_out,
                      void* stream) {
  if (!h || !hf || !e_out) return FMP_ERR_INVALID_ARG;
  const long long bytes = h->len * 8;
  if (fmp::overlap_bytes(hf, e_out, bytes)) return FMP_ERR_ALIAS;
  if (e_in && e_in != e_out && fmp::overlap_bytes(e_in, e_out, bytes)) return FMP_ERR_ALIAS;
  hipStream_t s = (hipStream_t)stream;
  for (const DomainDev& D : h->doms) {
    const double sc = m * 2.0 * std::sqrt(D.c);
    hipLaunchKernelGGL(fmp::k_curl_h, fmp::cell_grid(D), dim3(fmp::kFX, fmp::kFY), 0, s, hf, e_in,
                       sc, e_out, D, (const double*)h->d_eps);
    if (fmp_status st = fmp::hip_status(h, hipGetLastError(), "k_curl_h")) return st;
  }
  return FMP_OK;
}

fmp_status fmp_cn_workspace(fmp_handle h, const fmp_solve_opts* opts, size_t* bytes) {
  if (!h || !opts || !bytes) return FMP_ERR_INVALID_ARG;
  size_t solve = 0;
  if (fmp_status st = fmp_solve_workspace(h, opts, &solve)) return st;
  *bytes = fmp::align_cn(solve) + 2 * fmp::align_cn((size_t)h->len * 8);
  return FMP_OK;
}

fmp_status fmp_cn_step(fmp_handle h, double* E, double* H, const fmp_solve_opts* opts, void* ws,
                       size_t ws_bytes, fmp_solve_info* info, void* stream) {
  if (!h || !E || !H || !opts || !ws) return FMP_ERR_INVALID_ARG;
  const long long bytes = h->len * 8;
  if (fmp::overlap_bytes(E, H, bytes)) return FMP_ERR_ALIAS;
  size_t need = 0, solve = 0;
  if (fmp_status st = fmp_cn_workspace(h, opts, &need)) return st;
  if (ws_bytes < need || ((uintptr_t)ws) % fmp::kAlignCN) return FMP_ERR_WORKSPACE;
  fmp_solve_workspace(h, opts, &solve);
  char* base = (char*)ws;
  double* R = (double*)(base + fmp::align_cn(solve));
  double* X = (double*)(base + fmp::align_cn(solve) + fmp::align_cn((size_t)bytes));
  if (fmp::overlap_bytes(R, E, bytes) || fmp::overlap_bytes(R, H, bytes) ||
      fmp::overlap_bytes(X, E, bytes) || fmp::overlap_bytes(X, H, bytes))
    return FMP_ERR_ALIAS;
  hipStream_t s = (hipStream_t)stream;
  fmp_status st;
  // R = E + dt eps^-1 C^T (H - (dt/4) C E), with X holding the face vector
  if ((st = fmp_curl_e(h, E, nullptr, H, 1.0, -0.25, X, stream))) return st;
  if ((st = fmp_curl_h(h, X, E, 1.0, R, stream))) return st;
  // A E+ = R from the initial guess E
  if ((st = fmp::hip_status(h, hipMemcpyAsync(X, E, bytes, hipMemcpyDeviceToDevice, s),
                            "copy of the initial guess")))
    return st;
  const fmp_status sst = fmp_solve(h, R, X, opts, ws, solve, info, stream);
  if (sst != FMP_OK && sst != FMP_NOT_CONVERGED) return sst;
  // H+ = H - (dt/2) C (E+ + E), then E = E+
  if ((st = fmp_curl_e(h, X, E, H, 1.0, -0.5, H, stream))) return st;
  if ((st = fmp::hip_status(h, hipMemcpyAsync(E, X, bytes, hipMemcpyDeviceToDevice, s),
                            "copy of the new field")))
    return st;
  if ((st = fmp::hip_status(h, hipStreamSynchronize(s), "cn step"))) return st;
  return sst;
}

}  // extern "C"
