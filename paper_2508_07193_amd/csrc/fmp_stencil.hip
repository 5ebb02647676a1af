// Double-curl stencil y = A x = x + c diag(1/eps_e) K x on Yee grids with PEC walls.
//
// K = C^T C is the discrete double-curl of Sec. III-A (the curl display,
// eq. (6), and the matrix M; the (1,3) block and curl row 2 read with their
// typos fixed).  Written out per unknown it is a 13-point stencil; for E_x at
// (i+1/2, j, k):
//   (K E)_x = 4 Ex - Ex(j+1) - Ex(j-1) - Ex(k+1) - Ex(k-1)
//           + Ey(i+1, j+1/2) - Ey(i, j+1/2) - Ey(i+1, j-1/2) + Ey(i, j-1/2)
//           + Ez(i+1, k+1/2) - Ez(i, k+1/2) - Ez(i+1, k-1/2) + Ez(i, k-1/2)
// and the E_y, E_z rows follow by the cyclic relabelling x -> y -> z -> x.
// Values outside the domain or on a wall slot are zero.
//
// Mapping: a 64 x 4 tile of (i, j) columns per workgroup marches over 16
// z-planes.  Each lane keeps the values of its own column at k-1, k, k+1 in
// registers; in-plane neighbours come through L1/L2 (their owners load the
// same lines in the same step).  HBM traffic is then close to the algorithmic
// 8 bytes in + 8 bytes out per unknown.
#include "fmp_common.h"

namespace fmp {
namespace {

struct Dims {
  int nx, ny, nz;
  long long cs;  // component stride nz*ny*nx
};

template <int Q>
__device__ __forceinline__ double ld(const double* __restrict__ b, const Dims& d, int k, int j,
                                     int i) {
  if (i < 0 || j < 0 || k < 0 || i >= d.nx || j >= d.ny || k >= d.nz) return 0.0;
  // the two node axes of component Q hold the wall in slot 0
  if (Q == 0 && (j == 0 || k == 0)) return 0.0;
  if (Q == 1 && (i == 0 || k == 0)) return 0.0;
  if (Q == 2 && (i == 0 || j == 0)) return 0.0;
  return b[Q * d.cs + ((long long)k * d.ny + j) * d.nx + i];
}

__device__ __forceinline__ double cell_eps(const double* __restrict__ e, const DomainDev& D, int i,
                                           int j, int k) {
  const int b = D.eps_b;
  return e[D.eps_off + ((k / b) * D.eps_nby + (j / b)) * D.eps_nbx + (i / b)];
}

__global__ __launch_bounds__(256) void k_curlcurl(const double* __restrict__ x,
                                                  double* __restrict__ y,
                                                  const DomainDev* __restrict__ doms,
                                                  const StencilTile* __restrict__ tiles,
                                                  const double* __restrict__ eps) {
  const StencilTile T = tiles[blockIdx.x];
  const DomainDev D = doms[T.dom];
  const int i = T.x0 + (int)(threadIdx.x % kStencilTX);
  const int j = T.y0 + (int)(threadIdx.x / kStencilTX);
  if (i >= D.nx || j >= D.ny) return;
  const Dims d{D.nx, D.ny, D.nz, (long long)D.nz * D.ny * D.nx};
  const double* xb = x + D.offset;
  double* yb = y + D.offset;
  const int k0 = T.z0, k1 = min(T.z0 + kStencilZC, D.nz);

  // rolling own-column values
  double exm = ld<0>(xb, d, k0 - 1, j, i), ex0 = ld<0>(xb, d, k0, j, i);
  double eym = ld<1>(xb, d, k0 - 1, j, i), ey0 = ld<1>(xb, d, k0, j, i);
  double ezm = ld<2>(xb, d, k0 - 1, j, i);
  for (int k = k0; k < k1; ++k) {
    const double exp1 = ld<0>(xb, d, k + 1, j, i);
    const double eyp1 = ld<1>(xb, d, k + 1, j, i);
    const double ez0 = ld<2>(xb, d, k, j, i);

    // E_x row at (i+1/2, j, k)
    const double kx = 4.0 * ex0 - ld<0>(xb, d, k, j + 1, i) - ld<0>(xb, d, k, j - 1, i) - exp1 -
                      exm + (ld<1>(xb, d, k, j, i + 1) - ey0 - ld<1>(xb, d, k, j - 1, i + 1) +
                             ld<1>(xb, d, k, j - 1, i)) +
                      (ld<2>(xb, d, k, j, i + 1) - ez0 - ld<2>(xb, d, k - 1, j, i + 1) + ezm);
    // E_y row at (i, j+1/2, k)
    const double ky = 4.0 * ey0 - eyp1 - eym - ld<1>(xb, d, k, j, i + 1) -
                      ld<1>(xb, d, k, j, i - 1) +
                      (ld<2>(xb, d, k, j + 1, i) - ez0 - ld<2>(xb, d, k - 1, j + 1, i) + ezm) +
                      (ld<0>(xb, d, k, j + 1, i) - ex0 - ld<0>(xb, d, k, j + 1, i - 1) +
                       ld<0>(xb, d, k, j, i - 1));
    // E_z row at (i, j, k+1/2)
    const double kz = 4.0 * ez0 - ld<2>(xb, d, k, j, i + 1) - ld<2>(xb, d, k, j, i - 1) -
                      ld<2>(xb, d, k, j + 1, i) - ld<2>(xb, d, k, j - 1, i) +
                      (exp1 - ex0 - ld<0>(xb, d, k + 1, j, i - 1) + ld<0>(xb, d, k, j, i - 1)) +
                      (eyp1 - ey0 - ld<1>(xb, d, k + 1, j - 1, i) + ld<1>(xb, d, k, j - 1, i));

    double sx = D.c, sy = D.c, sz = D.c;
    if (D.eps_b > 0) {
      // edge permittivity: mean of the four cells sharing the edge, summed
      // in the order (-,-), (+,-), (-,+), (+,+) of the two transverse axes
      if (j >= 1 && k >= 1) {
        const double e = 0.25 * (((cell_eps(eps, D, i, j - 1, k - 1) + cell_eps(eps, D, i, j - 1, k)) +
                                  cell_eps(eps, D, i, j, k - 1)) + cell_eps(eps, D, i, j, k));
        sx = D.c / e;
      }
      if (i >= 1 && k >= 1) {
        const double e = 0.25 * (((cell_eps(eps, D, i - 1, j, k - 1) + cell_eps(eps, D, i - 1, j, k)) +
                                  cell_eps(eps, D, i, j, k - 1)) + cell_eps(eps, D, i, j, k));
        sy = D.c / e;
      }
      if (i >= 1 && j >= 1) {
        const double e = 0.25 * (((cell_eps(eps, D, i - 1, j - 1, k) + cell_eps(eps, D, i - 1, j, k)) +
                                  cell_eps(eps, D, i, j - 1, k)) + cell_eps(eps, D, i, j, k));
        sz = D.c / e;
      }
    }
    const long long o = ((long long)k * D.ny + j) * D.nx + i;
    yb[o] = (j == 0 || k == 0) ? 0.0 : ex0 + sx * kx;
    yb[d.cs + o] = (i == 0 || k == 0) ? 0.0 : ey0 + sy * ky;
    yb[2 * d.cs + o] = (i == 0 || j == 0) ? 0.0 : ez0 + sz * kz;

    exm = ex0; ex0 = exp1;
    eym = ey0; ey0 = eyp1;
    ezm = ez0;
  }
}

}  // namespace

hipError_t launch_curlcurl(const double* x, double* y, const DomainDev* doms,
                           const StencilTile* tiles, int ntiles, const double* eps,
                           hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_curlcurl, dim3(ntiles), dim3(kStencilTX * kStencilTY), 0, s, x, y, doms,
                     tiles, eps);
  return hipGetLastError();
}

}  // namespace fmp
