// Exact PEC-box solves of the RAS preconditioner on the vector ALU (FP64 / FP32).
//
// Per box and component (Sec. III-A Steps 1-3; Algorithm 1, exact_solve):
//   forward transform G: DCT-II along the component's own axis, DST-I along
//   the two node axes (the closed-form singular vectors of the 1-D difference
//   for a PEC box), then at each wavenumber (p, q, r) the 3x3 solve of
//   eq. (12), written in closed form (Sherman-Morrison):
//       e = (r + alpha s (s . r)) / (1 + alpha |s|^2),  s = (sigma_p, sigma_q, sigma_r),
//   then the inverse transform G^T.  The reorderings P, P^T of Step 2 are
//   never materialised: the solve reads the three components of a wavenumber
//   from LDS.
//
// Three passes per batch of boxes, with the spectral staging W in HBM (or the
// last-level cache when a batch fits):
//   A  gather (RAS restriction S^gamma) + x and y forward contractions, per z-slab
//   B  z forward contraction + block solve + z inverse contraction, per column set
//   C  y and x inverse contractions + scatter of owned unknowns (S^0T) [+ coarse add]
//
// Contractions keep one pencil per lane in registers (length NP, the size
// class) and read the transform matrix through the scalar unit: every lane of
// a wave multiplies by the same matrix entry, so each FMA takes one SGPR
// operand and the matrix costs no vector registers or LDS bandwidth.
#include "fmp_common.h"

namespace fmp {
namespace {

template <typename T>
__device__ __forceinline__ T fmaT(T a, T b, T c) {
  return a * b + c;
}
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// Contraction out[p] = sum_l M[p][l] v[l] for p < n_out, each result handed to
// store(p, value).  M is row-major with stride kTS (the forward matrix for a
// forward transform, the transposed table for an inverse one), so a row is a
// contiguous run of scalar loads.  The output loop stays rolled: one row of M
// lives in SGPRs at a time (fully unrolling it makes the compiler hoist every
// row and spill SGPRs into VGPR lanes).  Two accumulators halve the FMA chain.
template <typename T, int NP, class Store>
__device__ __forceinline__ void contract(const T* __restrict__ M, const T (&v)[NP], int n_out,
                                         Store store) {
#pragma unroll 1
  for (int p = 0; p < n_out; ++p) {
    const T* __restrict__ row = M + p * kTS;
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int l = 0; l + 1 < NP; l += 2) {
      a0 = fmaT<T>(row[l], v[l], a0);
      a1 = fmaT<T>(row[l + 1], v[l + 1], a1);
    }
    if (NP & 1) a0 = fmaT<T>(row[NP - 1], v[NP - 1], a0);
    store(p, a0 + a1);
  }
}

template <typename T>
__device__ __forceinline__ T recip(T d) {
  return T(1) / d;
}
// 1/d for d >= 1 from the hardware estimate and two Newton steps
template <>
__device__ __forceinline__ double recip<double>(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  return r;
}

// slot 0 of a component's node axes is the box wall
__device__ __forceinline__ bool box_wall(int q, int x, int y, int z) {
  return q == 0 ? (y == 0 || z == 0) : (q == 1 ? (x == 0 || z == 0) : (x == 0 || y == 0));
}

template <int NP>
constexpr int zslab() {
  return 256 / NP;
}

// ---------------------------------------------------------------- pass A
template <typename T, int NP>
__global__ __launch_bounds__(256) void k_pass_a(const double* __restrict__ r, T* __restrict__ W,
                                                const BoxDev* __restrict__ boxes,
                                                const DomainDev* __restrict__ doms,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab) {
  constexpr int ZS = zslab<NP>();
  __shared__ T buf[ZS][NP][NP + 1];
  const int4 wk = work[blockIdx.x];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const int plane = ny * nx;
  const int tot = nzs * plane;
  const int t = threadIdx.x;

  for (int e = t; e < tot; e += 256) {          // S^gamma: gather the slab
    const int zl = e / plane;
    const int rem = e - zl * plane;
    const int y = rem / nx;
    const int x = rem - y * nx;
    const int lz = z0 + zl;
    T val = T(0);
    if (!box_wall(q, x, y, lz))
      val = (T)src[((long long)(B.bz0 + lz) * D.ny + (B.by0 + y)) * D.nx + (B.bx0 + x)];
    buf[zl][y][x] = val;
  }
  __syncthreads();

  T v[NP];
  const T* Tx = tab + (q == 0 ? B.dct[0] : B.dst[0]);
  if (t < nzs * ny) {                             // x contraction, one row per lane
    const int zl = t / ny, y = t - zl * ny;
#pragma unroll
    for (int l = 0; l < NP; ++l) v[l] = (l < nx) ? buf[zl][y][l] : T(0);
    contract<T, NP>(Tx, v, nx, [&](int p, T val) { buf[zl][y][p] = val; });
  }
  __syncthreads();

  const T* Ty = tab + (q == 1 ? B.dct[1] : B.dst[1]);
  if (t < nzs * nx) {                             // y contraction, one column per lane
    const int zl = t / nx, x = t - zl * nx;
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = (m < ny) ? buf[zl][m][x] : T(0);
    T* dst = W + B.w_off + (long long)q * B.vol + (long long)(z0 + zl) * plane + x;
    contract<T, NP>(Ty, v, ny, [&](int p, T val) { dst[p * nx] = val; });
  }
}

// ---------------------------------------------------------------- pass B
template <typename T, int NP>
__global__ __launch_bounds__(192) void k_pass_b(T* __restrict__ W, const BoxDev* __restrict__ boxes,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab) {
  __shared__ T ex[3][NP][64];
  const int4 wk = work[blockIdx.x];
  const BoxDev& B = boxes[wk.x];
  // one wave per component; readfirstlane tells the compiler q is wave-uniform,
  // so the matrix entries below stay scalar operands
  const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int plane = ny * nx;
  const int c = wk.y + lane;
  const bool active = c < plane;
  T* col = W + B.w_off + (long long)q * B.vol + (active ? c : 0);

  T v[NP];
#pragma unroll
  for (int l = 0; l < NP; ++l) v[l] = (active && l < nz) ? col[(long long)l * plane] : T(0);
  const bool own = q == 2;                        // DCT-II along z for E_z, DST-I otherwise
  const T* Tz = tab + (own ? B.dct[2] : B.dst[2]);
  const T* TzT = tab + (own ? B.dctT[2] : B.dst[2]);
  contract<T, NP>(Tz, v, NP, [&](int r, T val) { ex[q][r][lane] = val; });
  __syncthreads();

  const int yy = active ? c / nx : 0;
  const int xx = active ? c - yy * nx : 0;
  const T sx = tab[B.sig[0] + xx];
  const T sy = tab[B.sig[1] + yy];
  const T* sz = tab + B.sig[2];
  const T alpha = (T)B.alpha;
  const T sxy2 = fmaT<T>(sx, sx, sy * sy);
#pragma unroll
  for (int rr = 0; rr < NP; ++rr) {               // e = (r + alpha s (s.r)) / (1 + alpha |s|^2)
    const T s3 = sz[rr];
    const T a = ex[0][rr][lane], b = ex[1][rr][lane], d = ex[2][rr][lane];
    const T dot = fmaT<T>(sx, a, fmaT<T>(sy, b, s3 * d));
    const T sq = q == 0 ? sx : (q == 1 ? sy : s3);
    const T rq = q == 0 ? a : (q == 1 ? b : d);
    v[rr] = fmaT<T>(alpha * sq, dot, rq) * recip<T>(fmaT<T>(alpha, fmaT<T>(s3, s3, sxy2), T(1)));
  }
  if (active)
    contract<T, NP>(TzT, v, nz, [&](int l, T val) { col[(long long)l * plane] = val; });
}

// ---------------------------------------------------------------- pass C
template <typename T, int NP>
__global__ __launch_bounds__(256) void k_pass_c(const T* __restrict__ W, double* __restrict__ z,
                                                const BoxDev* __restrict__ boxes,
                                                const DomainDev* __restrict__ doms,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ coarse, int nsub) {
  constexpr int ZS = zslab<NP>();
  __shared__ T buf[ZS][NP][NP + 1];
  const int4 wk = work[blockIdx.x];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int plane = ny * nx;
  const int tot = nzs * plane;
  const int t = threadIdx.x;
  const T* srcw = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;

  for (int e = t; e < tot; e += 256) {
    const int zl = e / plane;
    const int rem = e - zl * plane;
    const int y = rem / nx;
    const int x = rem - y * nx;
    buf[zl][y][x] = srcw[e];
  }
  __syncthreads();

  T v[NP];
  const T* TyT = tab + (q == 1 ? B.dctT[1] : B.dst[1]);
  if (t < nzs * nx) {                             // y inverse, one column per lane
    const int zl = t / nx, x = t - zl * nx;
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = (m < ny) ? buf[zl][m][x] : T(0);
    contract<T, NP>(TyT, v, ny, [&](int m, T val) { buf[zl][m][x] = val; });
  }
  __syncthreads();
  const T* TxT = tab + (q == 0 ? B.dctT[0] : B.dst[0]);
  if (t < nzs * ny) {                             // x inverse, one row per lane
    const int zl = t / ny, y = t - zl * ny;
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = (p < nx) ? buf[zl][y][p] : T(0);
    contract<T, NP>(TxT, v, nx, [&](int l, T val) { buf[zl][y][l] = val; });
  }
  __syncthreads();

  // S^0T: write the owned part of the slab
  const int lz0 = max(z0, B.oz0 - B.bz0), lz1 = min(z0 + nzs, B.oz0 - B.bz0 + B.sz);
  if (lz1 <= lz0) return;
  const int ly0 = B.oy0 - B.by0, lx0 = B.ox0 - B.bx0;
  const int oplane = B.sy * B.sx;
  const int otot = (lz1 - lz0) * oplane;
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const double cq = coarse ? coarse[(long long)q * nsub + B.sub] : 0.0;
  for (int e = t; e < otot; e += 256) {
    const int zl = e / oplane;
    const int rem = e - zl * oplane;
    const int y = rem / B.sx;
    const int x = rem - y * B.sx;
    const int lz = lz0 + zl, ly = ly0 + y, lx = lx0 + x;
    const int gz = B.bz0 + lz, gy = B.by0 + ly, gx = B.bx0 + lx;
    double val = (double)buf[lz - z0][ly][lx];
    if (coarse && !box_wall(q, gx, gy, gz)) val += cq;
    dst[((long long)gz * D.ny + gy) * D.nx + gx] = val;
  }
}

template <typename T, int NP>
hipError_t run_a(const double* r, void* W, const BoxDev* boxes, const DomainDev* doms,
                 const int4* work, int nwork, const void* tab, hipStream_t s) {
  hipLaunchKernelGGL((k_pass_a<T, NP>), dim3(nwork), dim3(256), 0, s, r, (T*)W, boxes, doms, work,
                     (const T*)tab);
  return hipGetLastError();
}
template <typename T, int NP>
hipError_t run_b(void* W, const BoxDev* boxes, const int4* work, int nwork, const void* tab,
                 hipStream_t s) {
  hipLaunchKernelGGL((k_pass_b<T, NP>), dim3(nwork), dim3(192), 0, s, (T*)W, boxes, work,
                     (const T*)tab);
  return hipGetLastError();
}
template <typename T, int NP>
hipError_t run_c(const void* W, double* z, const BoxDev* boxes, const DomainDev* doms,
                 const int4* work, int nwork, const void* tab, const double* coarse, int nsub,
                 hipStream_t s) {
  hipLaunchKernelGGL((k_pass_c<T, NP>), dim3(nwork), dim3(256), 0, s, (const T*)W, z, boxes, doms,
                     work, (const T*)tab, coarse, nsub);
  return hipGetLastError();
}

#define FMP_CLASS_SWITCH(CLS, CALL)                     \
  switch (CLS) {                                        \
    case 0: return CALL(8);                             \
    case 1: return CALL(16);                            \
    case 2: return CALL(24);                            \
    case 3: return CALL(26);                            \
    case 4: return CALL(32);                            \
    case 5: return CALL(34);                            \
    case 6: return CALL(40);                            \
    case 7: return CALL(48);                            \
    default: return hipErrorInvalidValue;               \
  }

}  // namespace

int pass_a_zslab(int cls) { return 256 / kClasses[cls]; }

hipError_t launch_pass_a(int prec, int cls, const double* r, void* W, const BoxDev* boxes,
                         const DomainDev* doms, const int4* work, int nwork, const void* tab,
                         hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (prec == 0) {
#define CALL(N) run_a<double, N>(r, W, boxes, doms, work, nwork, tab, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  } else {
#define CALL(N) run_a<float, N>(r, W, boxes, doms, work, nwork, tab, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  }
}

hipError_t launch_pass_b(int prec, int cls, void* W, const BoxDev* boxes, const int4* work,
                         int nwork, const void* tab, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (prec == 0) {
#define CALL(N) run_b<double, N>(W, boxes, work, nwork, tab, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  } else {
#define CALL(N) run_b<float, N>(W, boxes, work, nwork, tab, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  }
}

hipError_t launch_pass_c(int prec, int cls, const void* W, double* z, const BoxDev* boxes,
                         const DomainDev* doms, const int4* work, int nwork, const void* tab,
                         const double* coarse, int nsub, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (prec == 0) {
#define CALL(N) run_c<double, N>(W, z, boxes, doms, work, nwork, tab, coarse, nsub, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  } else {
#define CALL(N) run_c<float, N>(W, z, boxes, doms, work, nwork, tab, coarse, nsub, s)
    FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  }
}

}  // namespace fmp
