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
// Mapping: a workgroup owns a 64 x TY tile of (i, j) columns and marches over
// kStencilZC = 64 z-planes; TY is 4, 8 or 16 (256, 512 or 1024 threads),
// chosen by fmp_autotune (8 by default, the fastest of the shapes swept at
// 256^3).
// Three rolling LDS planes (k-1, k, k+1) of all three components, with a
// one-cell halo in x and y, are filled by coalesced loads
// that zero wall slots and out-of-domain cells once, so the stencil itself
// reads LDS without bounds checks.  Cell permittivities of planes k-1 and k
// are staged the same way.  HBM sees each value once (halos come from L2),
// i.e. the algorithmic 8 bytes in + 8 bytes out per unknown.
//
// Tiles are enumerated x fastest, then y, then z; the block index is
// remapped so that each XCD (blocks are dealt to the 8 XCDs round-robin)
// works on a contiguous run of tiles and finds their halos in its own L2.
#include "fmp_common.h"

namespace fmp {
namespace {

// 1/d for d > 0 (a sum of four permittivities): hardware estimate, two Newton steps
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  return r;
}

constexpr int TX = kStencilTX;
constexpr int HX = TX + 2;                // tile with halo in x

template <int TY>
__global__ __launch_bounds__(TX * TY) void k_curlcurl(const double* __restrict__ x,
                                                      double* __restrict__ y,
                                                      const DomainDev* __restrict__ doms,
                                                      const StencilTile* __restrict__ tiles,
                                                      int ntiles, const double* __restrict__ eps) {
  constexpr int HY = TY + 2;                  // tile with halo in y
  __shared__ double P[3][3][HY][HX];          // [slot][component][j][i]
  __shared__ double E[2][TY + 1][TX + 1];     // cell eps, [slot][j][i] for cells j0-1.., i0-1..
  const StencilTile T = tiles[xcd_remap(blockIdx.x, ntiles)];
  const DomainDev D = doms[T.dom];
  const int nx = D.nx, ny = D.ny, nz = D.nz;
  const long long cs = (long long)nz * ny * nx;
  const double* __restrict__ xb = x + D.offset;
  double* __restrict__ yb = y + D.offset;
  const int t = threadIdx.x;
  const int tx = t % TX, ty = t / TX;
  const int i = T.x0 + tx, j = T.y0 + ty;
  const int k0 = T.z0, k1 = min(T.z0 + kStencilZC, nz);
  const bool use_eps = D.eps_b > 0;

  // Plane staging is software-pipelined: a thread holds its share of plane
  // k+2 (and of the cell-eps plane k+1) in registers, loaded while plane k is
  // being computed, and commits it to LDS after the step's barrier.
  constexpr int NE = (3 * HY * HX + TX * TY - 1) / (TX * TY);
  constexpr int NEE = ((TY + 1) * (TX + 1) + TX * TY - 1) / (TX * TY);
  double pre[NE], epre[NEE];
  unsigned ok_mask = 0;
  auto fetch = [&](int kk) {
    static_assert(NE <= 32, "validity flags are kept in one 32-bit mask");
    ok_mask = 0;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = min(t + i * TX * TY, 3 * HY * HX - 1);
      const int q = e / (HY * HX);
      const int rem = e - q * (HY * HX);
      const int jj = rem / HX, ii = rem - jj * HX;
      const int gi = T.x0 - 1 + ii, gj = T.y0 - 1 + jj;
      bool ok = gi >= 0 && gj >= 0 && kk >= 0 && gi < nx && gj < ny && kk < nz;
      if (q == 0) ok = ok && gj != 0 && kk != 0;
      else if (q == 1) ok = ok && gi != 0 && kk != 0;
      else ok = ok && gi != 0 && gj != 0;
      if (ok) ok_mask |= 1u << i;
      const int ci = min(max(gi, 0), nx - 1), cj = min(max(gj, 0), ny - 1);
      const int ck = min(max(kk, 0), nz - 1);
      pre[i] = xb[q * cs + ((long long)ck * ny + cj) * nx + ci];
    }
  };
  auto commit = [&](int s) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = t + i * TX * TY;
      if (e < 3 * HY * HX) (&P[s][0][0][0])[e] = ((ok_mask >> i) & 1u) ? pre[i] : 0.0;
    }
  };
  auto fetch_eps = [&](int kk) {
    const int b = D.eps_b;
#pragma unroll
    for (int i = 0; i < NEE; ++i) {
      const int e = min(t + i * TX * TY, (TY + 1) * (TX + 1) - 1);
      const int jj = e / (TX + 1), ii = e - jj * (TX + 1);
      const int gi = min(max(T.x0 - 1 + ii, 0), nx - 1);
      const int gj = min(max(T.y0 - 1 + jj, 0), ny - 1);
      const int gk = min(max(kk, 0), nz - 1);
      epre[i] = eps[D.eps_off + ((gk / b) * D.eps_nby + (gj / b)) * D.eps_nbx + (gi / b)];
    }
  };
  auto commit_eps = [&](int s) {
#pragma unroll
    for (int i = 0; i < NEE; ++i) {
      const int e = t + i * TX * TY;
      if (e < (TY + 1) * (TX + 1)) (&E[s][0][0])[e] = epre[i];
    }
  };

  fetch(k0 - 1);
  commit((k0 + 2) % 3);
  fetch(k0);
  commit(k0 % 3);
  if (use_eps) {
    fetch_eps(k0 - 1);
    commit_eps((k0 + 1) & 1);
    fetch_eps(k0);
  }
  fetch(k0 + 1);
  for (int k = k0; k < k1; ++k) {
    commit((k + 1) % 3);
    if (use_eps) commit_eps(k & 1);
    __syncthreads();
    if (k + 1 < k1) {                            // prefetch the next step's planes
      fetch(k + 2);
      if (use_eps) fetch_eps(k + 1);
    }
    const int sm = (k + 2) % 3, s0 = k % 3, sp = (k + 1) % 3;
    const int a = ty + 1, c = tx + 1;      // own position inside the halo tile
    const double ex0 = P[s0][0][a][c], ey0 = P[s0][1][a][c], ez0 = P[s0][2][a][c];
    const double kx = 4.0 * ex0 - P[s0][0][a + 1][c] - P[s0][0][a - 1][c] - P[sp][0][a][c] -
                      P[sm][0][a][c] +
                      (P[s0][1][a][c + 1] - ey0 - P[s0][1][a - 1][c + 1] + P[s0][1][a - 1][c]) +
                      (P[s0][2][a][c + 1] - ez0 - P[sm][2][a][c + 1] + P[sm][2][a][c]);
    const double ky = 4.0 * ey0 - P[sp][1][a][c] - P[sm][1][a][c] - P[s0][1][a][c + 1] -
                      P[s0][1][a][c - 1] +
                      (P[s0][2][a + 1][c] - ez0 - P[sm][2][a + 1][c] + P[sm][2][a][c]) +
                      (P[s0][0][a + 1][c] - ex0 - P[s0][0][a + 1][c - 1] + P[s0][0][a][c - 1]);
    const double kz = 4.0 * ez0 - P[s0][2][a][c + 1] - P[s0][2][a][c - 1] - P[s0][2][a + 1][c] -
                      P[s0][2][a - 1][c] +
                      (P[sp][0][a][c] - ex0 - P[sp][0][a][c - 1] + P[s0][0][a][c - 1]) +
                      (P[sp][1][a][c] - ey0 - P[sp][1][a - 1][c] + P[s0][1][a - 1][c]);
    double sx = D.c, sy = D.c, sz = D.c;
    if (use_eps) {
      // edge permittivity: mean of the four cells sharing the edge, summed in
      // the order (-,-), (+,-), (-,+), (+,+) of the two transverse axes;
      // c / mean = 4c / sum, the reciprocal from the hardware estimate and
      // two Newton steps (within an ulp or two of the division)
      const int em = (k + 1) & 1, e0 = k & 1;   // cell planes k-1 and k
      const int ja = ty + 1, ia = tx + 1;       // cell (j, i) inside the eps tile
      const double c4 = 4.0 * D.c;
      sx = c4 * recip(((E[em][ja - 1][ia] + E[e0][ja - 1][ia]) + E[em][ja][ia]) + E[e0][ja][ia]);
      sy = c4 * recip(((E[em][ja][ia - 1] + E[e0][ja][ia - 1]) + E[em][ja][ia]) + E[e0][ja][ia]);
      sz = c4 * recip(((E[e0][ja - 1][ia - 1] + E[e0][ja][ia - 1]) + E[e0][ja - 1][ia]) +
                      E[e0][ja][ia]);
    }
    if (i < nx && j < ny) {                      // y is not re-read here: streaming stores
      const long long o = ((long long)k * ny + j) * nx + i;
      __builtin_nontemporal_store((j == 0 || k == 0) ? 0.0 : ex0 + sx * kx, yb + o);
      __builtin_nontemporal_store((i == 0 || k == 0) ? 0.0 : ey0 + sy * ky, yb + cs + o);
      __builtin_nontemporal_store((i == 0 || j == 0) ? 0.0 : ez0 + sz * kz, yb + 2 * cs + o);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_curlcurl(int ty, const double* x, double* y, const DomainDev* doms,
                           const StencilTile* tiles, int ntiles, const double* eps,
                           hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  switch (ty) {
    case 4:
      hipLaunchKernelGGL(k_curlcurl<4>, dim3(ntiles), dim3(TX * 4), 0, s, x, y, doms, tiles,
                         ntiles, eps);
      break;
    case 8:
      hipLaunchKernelGGL(k_curlcurl<8>, dim3(ntiles), dim3(TX * 8), 0, s, x, y, doms, tiles,
                         ntiles, eps);
      break;
    case 16:
      hipLaunchKernelGGL(k_curlcurl<16>, dim3(ntiles), dim3(TX * 16), 0, s, x, y, doms, tiles,
                         ntiles, eps);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fmp
