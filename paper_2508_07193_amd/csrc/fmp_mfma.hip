// BF16 transform passes on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Same three-pass structure and the same mathematics as the vector-ALU passes
// (Sec. III-A Steps 1-3; Algorithm 1, exact_solve: forward DCT-II/DST-I per
// component, closed-form 3x3 solve of eq. (12) per wavenumber, inverse), but
// every directional contraction is a small GEMM on the matrix cores, the form
// the paper gives its transforms (Sec. III-C, GEMM-based discrete transform):
//   x-contraction of a z-slab: rows (z, y), K = x, N = p
//   y-contraction:             rows (z, p), K = y, N = q
//   z-contraction:             rows = 64 columns (y, x), K = z, N = r
// Operands are rounded to bf16 (inputs when a fragment is loaded, tables at
// setup), products accumulate in FP32, the block solve is FP32 and the staging
// between passes is bf16.
//
// Fragment layout (16x16x32): lane l holds A[m = l%16][k = 8(l/16) .. +7],
// B[k = 8(l/16) .. +7][n = l%16], and D[m = 4(l/16) + i][n = l%16], i < 4.
// The tables are stored transposed for the B operand, Bt[n][k] with row
// stride 64, so a lane's eight k values are one 16-byte load.
#include "fmp_common.h"

namespace fmp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kTB = 64;   // bf16 table row stride

// D[row0 .. row0+16)[0 .. n_out) = sum_k A[row][k] Bt[n][k] for one wave;
// A is read through aload(row, k) (0 outside), results go to dstore.
template <int KP, class ALoad, class DStore>
__device__ __forceinline__ void wave_gemm(int row0, int nrows, int n_out,
                                          const __bf16* __restrict__ Bt, ALoad aload,
                                          DStore dstore) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int row = row0 + r;
  bf16x8 a[KP / 32];
#pragma unroll
  for (int ks = 0; ks < KP / 32; ++ks)
#pragma unroll
    for (int j = 0; j < 8; ++j) a[ks][j] = (__bf16)(row < nrows ? aload(row, ks * 32 + 8 * g + j) : 0.f);
  for (int n0 = 0; n0 < n_out; n0 += 16) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int n = n0 + r;
#pragma unroll
    for (int ks = 0; ks < KP / 32; ++ks) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bt + n * kTB + ks * 32 + 8 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int rr = row0 + 4 * g + ii;
      if (rr < nrows && n < n_out) dstore(rr, n, acc[ii]);
    }
  }
}

__device__ __forceinline__ bool box_wall(int q, int x, int y, int z) {
  return q == 0 ? (y == 0 || z == 0) : (q == 1 ? (x == 0 || z == 0) : (x == 0 || y == 0));
}

// e / d for 0 <= e < 2^24 from a precomputed 1/d (see the vector-ALU passes)
__device__ __forceinline__ int qdiv(int e, double inv_d) { return (int)(((double)e + 0.5) * inv_d); }

template <int NP>
constexpr int zslab() {
  return 256 / NP;
}
template <int NP>
constexpr int kpad() {
  return NP <= 32 ? 32 : 64;
}

// The staging W between passes is bf16: every consumer rounds its MFMA
// operands to bf16 anyway, so this halves the traffic at no cost in accuracy.
// LDS slabs are dense [zl][y][x] (index = linear element id) in FP32.

// ---------------------------------------------------------------- pass A
template <int NP>
__global__ __launch_bounds__(256) void k_mpass_a(const double* __restrict__ r, __bf16* __restrict__ W,
                                                 const BoxDev* __restrict__ boxes,
                                                 const DomainDev* __restrict__ doms,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb) {
  constexpr int ZS = zslab<NP>(), KP = kpad<NP>();
  constexpr int MAXE = (ZS * NP * NP + 255) / 256;
  __shared__ float buf[ZS * NP * NP];
  __shared__ float obuf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const int plane = ny * nx, tot = nzs * plane;
  const int t = threadIdx.x, wave = t >> 6;
  const double inv_plane = 1.0 / plane, inv_nx = 1.0 / nx;
  double vals[MAXE];
  unsigned wall = 0;
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {
    const int e = min(t + 256 * i, tot - 1);
    const int zl = qdiv(e, inv_plane), rem = e - zl * plane;
    const int y = qdiv(rem, inv_nx), x = rem - y * nx;
    if (box_wall(q, x, y, z0 + zl)) wall |= 1u << i;
    vals[i] = src[((B.bz0 + z0 + zl) * D.ny + (B.by0 + y)) * D.nx + (B.bx0 + x)];
  }
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {
    const int e = t + 256 * i;
    if (e < tot) buf[e] = ((wall >> i) & 1u) ? 0.f : (float)vals[i];
  }
  __syncthreads();
  {  // x: rows rho = (zl, y) at buf[rho * nx], K = x, N = p
    const __bf16* Bt = tb + (q == 0 ? B.mdct[0] : B.mdst[0]);
    const int R = nzs * ny;
    for (int tile = wave; tile * 16 < R; tile += 4)
      wave_gemm<KP>(tile * 16, R, nx, Bt,
                    [&](int rho, int k) { return k < nx ? buf[rho * nx + k] : 0.f; },
                    [&](int rho, int p, float v) { obuf[rho * nx + p] = v; });
  }
  __syncthreads();
  {  // y: rows rho = (zl, p), K = y, N = q
    const __bf16* Bt = tb + (q == 1 ? B.mdct[1] : B.mdst[1]);
    const int R = nzs * nx;
    for (int tile = wave; tile * 16 < R; tile += 4)
      wave_gemm<KP>(tile * 16, R, ny, Bt,
                    [&](int rho, int k) {
                      const int zl = qdiv(rho, inv_nx), p = rho - zl * nx;
                      return k < ny ? obuf[zl * plane + k * nx + p] : 0.f;
                    },
                    [&](int rho, int qq, float v) {
                      const int zl = qdiv(rho, inv_nx), p = rho - zl * nx;
                      buf[zl * plane + qq * nx + p] = v;
                    });
  }
  __syncthreads();
  __bf16* dst = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;
  for (int e = t; e < tot; e += 256) dst[e] = (__bf16)buf[e];
}

// ---------------------------------------------------------------- pass B
template <int NP>
__global__ __launch_bounds__(256) void k_mpass_b(__bf16* __restrict__ W,
                                                 const BoxDev* __restrict__ boxes,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb,
                                                 const float* __restrict__ sig) {
  constexpr int KP = kpad<NP>();
  constexpr int MAXE = (3 * NP * 64 + 255) / 256;
  __shared__ float L[3][NP][64];
  __shared__ float X[3][NP][64];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int plane = ny * nx, c0 = wk.y;
  const int t = threadIdx.x, wave = t >> 6;
  const int n3 = 3 * nz * 64;
  float vals[MAXE];
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {                // column slab of the three components
    const int e = min(t + 256 * i, n3 - 1);
    const int q = e / (nz * 64), rem = e - q * nz * 64, l = rem >> 6, c = rem & 63;
    vals[i] = (float)W[B.w_off + q * B.vol + (long long)l * plane + min(c0 + c, plane - 1)];
  }
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {
    const int e = t + 256 * i;
    if (e < n3) {
      const int q = e / (nz * 64), rem = e - q * nz * 64, l = rem >> 6, c = rem & 63;
      L[q][l][c] = vals[i];
    }
  }
  __syncthreads();
  for (int task = wave; task < 12; task += 4) {        // forward z, 3 components x 4 row tiles
    const int q = task >> 2, tile = task & 3;
    const __bf16* Bt = tb + (q == 2 ? B.mdct[2] : B.mdst[2]);
    wave_gemm<KP>(tile * 16, 64, nz, Bt, [&](int c, int l) { return l < nz ? L[q][l][c] : 0.f; },
                  [&](int c, int rr, float v) { X[q][rr][c] = v; });
  }
  __syncthreads();
  const float alpha = (float)B.alpha;
  for (int e = t; e < nz * 64; e += 256) {             // e = (r + alpha s (s.r)) / (1 + alpha |s|^2)
    const int rr = e >> 6, c = e & 63, col = min(c0 + c, plane - 1);
    const int yy = col / nx, xx = col - yy * nx;
    const float sx = sig[B.sig[0] + xx], sy = sig[B.sig[1] + yy], sz = sig[B.sig[2] + rr];
    const float a = X[0][rr][c], b = X[1][rr][c], d = X[2][rr][c];
    const float dot = __builtin_fmaf(sx, a, __builtin_fmaf(sy, b, sz * d));
    const float inv = 1.f / __builtin_fmaf(alpha, __builtin_fmaf(sx, sx, __builtin_fmaf(sy, sy, sz * sz)), 1.f);
    const float ad = alpha * dot;
    X[0][rr][c] = __builtin_fmaf(ad, sx, a) * inv;
    X[1][rr][c] = __builtin_fmaf(ad, sy, b) * inv;
    X[2][rr][c] = __builtin_fmaf(ad, sz, d) * inv;
  }
  __syncthreads();
  for (int task = wave; task < 12; task += 4) {        // inverse z
    const int q = task >> 2, tile = task & 3;
    const __bf16* Bt = tb + (q == 2 ? B.mdctT[2] : B.mdst[2]);
    wave_gemm<KP>(tile * 16, 64, nz, Bt, [&](int c, int rr) { return rr < nz ? X[q][rr][c] : 0.f; },
                  [&](int c, int l, float v) { L[q][l][c] = v; });
  }
  __syncthreads();
  for (int e = t; e < n3; e += 256) {
    const int q = e / (nz * 64), rem = e - q * nz * 64, l = rem >> 6, c = rem & 63;
    if (c0 + c < plane) W[B.w_off + q * B.vol + (long long)l * plane + c0 + c] = (__bf16)L[q][l][c];
  }
}

// ---------------------------------------------------------------- pass C
template <int NP>
__global__ __launch_bounds__(256) void k_mpass_c(const __bf16* __restrict__ W, double* __restrict__ z,
                                                 const BoxDev* __restrict__ boxes,
                                                 const DomainDev* __restrict__ doms,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb,
                                                 const double* __restrict__ coarse, int nsub) {
  constexpr int ZS = zslab<NP>(), KP = kpad<NP>();
  constexpr int MAXE = (ZS * NP * NP + 255) / 256;
  __shared__ float buf[ZS * NP * NP];
  __shared__ float obuf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int plane = ny * nx, tot = nzs * plane;
  const int t = threadIdx.x, wave = t >> 6;
  const double inv_nx = 1.0 / nx;
  const __bf16* srcw = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;
  float vals[MAXE];
#pragma unroll
  for (int i = 0; i < MAXE; ++i) vals[i] = (float)srcw[min(t + 256 * i, tot - 1)];
#pragma unroll
  for (int i = 0; i < MAXE; ++i)
    if (t + 256 * i < tot) buf[t + 256 * i] = vals[i];
  __syncthreads();
  {  // y inverse: rows rho = (zl, p), K = q, N = m
    const __bf16* Bt = tb + (q == 1 ? B.mdctT[1] : B.mdst[1]);
    const int R = nzs * nx;
    for (int tile = wave; tile * 16 < R; tile += 4)
      wave_gemm<KP>(tile * 16, R, ny, Bt,
                    [&](int rho, int k) {
                      const int zl = qdiv(rho, inv_nx), p = rho - zl * nx;
                      return k < ny ? buf[zl * plane + k * nx + p] : 0.f;
                    },
                    [&](int rho, int m, float v) {
                      const int zl = qdiv(rho, inv_nx), p = rho - zl * nx;
                      obuf[zl * plane + m * nx + p] = v;
                    });
  }
  __syncthreads();
  {  // x inverse: rows rho = (zl, y) at obuf[rho * nx], K = p, N = l
    const __bf16* Bt = tb + (q == 0 ? B.mdctT[0] : B.mdst[0]);
    const int R = nzs * ny;
    for (int tile = wave; tile * 16 < R; tile += 4)
      wave_gemm<KP>(tile * 16, R, nx, Bt,
                    [&](int rho, int k) { return k < nx ? obuf[rho * nx + k] : 0.f; },
                    [&](int rho, int l, float v) { buf[rho * nx + l] = v; });
  }
  __syncthreads();
  const int lz0 = max(z0, B.oz0 - B.bz0), lz1 = min(z0 + nzs, B.oz0 - B.bz0 + B.sz);
  if (lz1 <= lz0) return;
  const int ly0 = B.oy0 - B.by0, lx0 = B.ox0 - B.bx0;
  const int oplane = B.sy * B.sx, otot = (lz1 - lz0) * oplane;
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const double cq = coarse ? coarse[(long long)q * nsub + B.sub] : 0.0;
  const double inv_op = 1.0 / oplane, inv_sx = 1.0 / B.sx;
  for (int e = t; e < otot; e += 256) {
    const int zl = qdiv(e, inv_op), rem = e - zl * oplane;
    const int y = qdiv(rem, inv_sx), x = rem - y * B.sx;
    const int lz = lz0 + zl, ly = ly0 + y, lx = lx0 + x;
    const int gz = B.bz0 + lz, gy = B.by0 + ly, gx = B.bx0 + lx;
    double val = (double)buf[(lz - z0) * plane + ly * nx + lx];
    if (coarse && !box_wall(q, gx, gy, gz)) val += cq;
    dst[(gz * D.ny + gy) * D.nx + gx] = val;
  }
}

#define FMP_CLASS_SWITCH(CLS, CALL)                     \
  switch (CLS) {                                        \
    case 0: CALL(8); break;                             \
    case 1: CALL(16); break;                            \
    case 2: CALL(24); break;                            \
    case 3: CALL(26); break;                            \
    case 4: CALL(32); break;                            \
    case 5: CALL(34); break;                            \
    case 6: CALL(40); break;                            \
    case 7: CALL(48); break;                            \
    default: return hipErrorInvalidValue;               \
  }

}  // namespace

int mfma_zslab(int cls) { return 256 / kClasses[cls]; }

hipError_t launch_mfma_pass_a(int cls, const double* r, void* Wv, const BoxDev* boxes,
                              const DomainDev* doms, const int4* work, int nwork,
                              const __hip_bfloat16* tab, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  const __bf16* tb = reinterpret_cast<const __bf16*>(tab);
  __bf16* W = reinterpret_cast<__bf16*>(Wv);
#define CALL(N) hipLaunchKernelGGL((k_mpass_a<N>), dim3(nwork), dim3(256), 0, s, r, W, boxes, doms, work, tb)
  FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_mfma_pass_b(int cls, void* Wv, const BoxDev* boxes, const int4* work,
                              int nwork, const __hip_bfloat16* tab, const float* sig,
                              hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  const __bf16* tb = reinterpret_cast<const __bf16*>(tab);
  __bf16* W = reinterpret_cast<__bf16*>(Wv);
#define CALL(N) hipLaunchKernelGGL((k_mpass_b<N>), dim3(nwork), dim3(256), 0, s, W, boxes, work, tb, sig)
  FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_mfma_pass_c(int cls, const void* Wv, double* z, const BoxDev* boxes,
                              const DomainDev* doms, const int4* work, int nwork,
                              const __hip_bfloat16* tab, const double* coarse, int nsub,
                              hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  const __bf16* tb = reinterpret_cast<const __bf16*>(tab);
  const __bf16* W = reinterpret_cast<const __bf16*>(Wv);
#define CALL(N) hipLaunchKernelGGL((k_mpass_c<N>), dim3(nwork), dim3(256), 0, s, W, z, boxes, doms, work, tb, coarse, nsub)
  FMP_CLASS_SWITCH(cls, CALL)
#undef CALL
  return hipGetLastError();
}

}  // namespace fmp
