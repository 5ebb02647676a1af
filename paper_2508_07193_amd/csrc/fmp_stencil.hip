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
// reads LDS without bounds checks.  Cell permittivities come from the block
// table through the cache, four per column and z-block (the table is
// constant on cubes of b^3 cells), so they take no LDS.  HBM sees each value
// once (halos come from L2), i.e. the algorithmic 8 bytes in + 8 bytes out
// per unknown.  (Tiles 128 or 256 wide and 64 x 12 tiles measured slower at
// 256^3: 0.180, 0.268 and 0.256 ms against 0.171 ms for 64 x 8.)
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
  // k+2 in registers, loaded while plane k is being computed, and commits it
  // to LDS after the step's barrier.
  constexpr int NE = (3 * HY * HX + TX * TY - 1) / (TX * TY);
  double pre[NE];
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

  // Cell permittivities of the four cells (j-1 | j, i-1 | i) around the
  // thread's column, at planes k-1 (em) and k (e0), read from the block
  // table (constant on cubes of b^3 cells) through the cache: the column's
  // block indices are fixed for the whole march, and new values are loaded
  // only when plane k enters another z-block.  Cells outside the domain take
  // the nearest cell's value (they only meet edges that are wall slots).
  double em[4] = {1.0, 1.0, 1.0, 1.0}, e0[4] = {1.0, 1.0, 1.0, 1.0};
  long long cix[4] = {0, 0, 0, 0};
  long long zstride = 0;
  int bcur = -1;
  if (use_eps) {
    const int b = D.eps_b;
    const int bim = min(max(i - 1, 0), nx - 1) / b, bi0 = min(max(i, 0), nx - 1) / b;
    const int bjm = min(max(j - 1, 0), ny - 1) / b, bj0 = min(max(j, 0), ny - 1) / b;
    cix[0] = D.eps_off + (long long)bjm * D.eps_nbx + bim;
    cix[1] = D.eps_off + (long long)bjm * D.eps_nbx + bi0;
    cix[2] = D.eps_off + (long long)bj0 * D.eps_nbx + bim;
    cix[3] = D.eps_off + (long long)bj0 * D.eps_nbx + bi0;
    zstride = (long long)D.eps_nby * D.eps_nbx;
  }
  auto zblock = [&](int kk) { return min(max(kk, 0), nz - 1) / D.eps_b; };
  auto load_eps = [&](int bk, double (&e)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) e[c] = eps[cix[c] + bk * zstride];
  };

  fetch(k0 - 1);
  commit((k0 + 2) % 3);
  fetch(k0);
  commit(k0 % 3);
  if (use_eps) {
    load_eps(zblock(k0 - 1), em);
    bcur = zblock(k0);
    load_eps(bcur, e0);
  }
  fetch(k0 + 1);
  for (int k = k0; k < k1; ++k) {
    commit((k + 1) % 3);
    __syncthreads();
    if (k + 1 < k1) fetch(k + 2);                // prefetch the next step's plane
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
      const double c4 = 4.0 * D.c;
      sx = c4 * recip(((em[1] + e0[1]) + em[3]) + e0[3]);   // cells (j-1|j, i), k-1|k
      sy = c4 * recip(((em[2] + e0[2]) + em[3]) + e0[3]);   // cells (j, i-1|i), k-1|k
      sz = c4 * recip(((e0[0] + e0[2]) + e0[1]) + e0[3]);   // cells (j-1|j, i-1|i), k
    }
    if (i < nx && j < ny) {                      // y is not re-read here: streaming stores
      const long long o = ((long long)k * ny + j) * nx + i;
      __builtin_nontemporal_store((j == 0 || k == 0) ? 0.0 : ex0 + sx * kx, yb + o);
      __builtin_nontemporal_store((i == 0 || k == 0) ? 0.0 : ey0 + sy * ky, yb + cs + o);
      __builtin_nontemporal_store((i == 0 || j == 0) ? 0.0 : ez0 + sz * kz, yb + 2 * cs + o);
    }
    if (use_eps && k + 1 < k1) {                 // planes k, k+1 for the next step
#pragma unroll
      for (int c = 0; c < 4; ++c) em[c] = e0[c];
      const int bn = zblock(k + 1);
      if (bn != bcur) {
        bcur = bn;
        load_eps(bcur, e0);
      }
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
