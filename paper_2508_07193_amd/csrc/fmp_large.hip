// Exact PEC-box solves of large boxes (sides 49..96) in FP64 / FP32.
//
// The same mathematics as the three-pass path (Sec. III-A Steps 1-3;
// Algorithm 1, exact_solve: DCT-II along a component's own axis, DST-I along
// its node axes, the closed-form 3x3 solve of eq. (12), the transposed
// transforms), with every directional contraction done as the GEMM the paper
// writes it as (Sec. III-C): for a box component and an axis of length N,
//     Out[i][c] = sum_k T[i][k] In[k][c],
// T the N x N transform matrix and c running over the N^2 pencils, split by
// the even/odd symmetry of DCT-II / DST-I into two GEMMs of half the depth
// (the butterfly of the vector-ALU passes, one level deep: half the
// multiply-adds).  Pencils of these sizes do not fit one lane's registers
// with the table rows as scalar operands, so each contraction is a tiled
// GEMM through LDS: a 256-thread workgroup computes a 64 x 64 output tile
// (4 x 4 per thread) in steps of 16 along k.  The box staging holds two
// copies of each box (ping-pong between contractions):
//   gather (S^gamma r, walls 0) -> x, y, z forward -> solve -> z, y, x inverse
//   -> scatter of the owned unknowns (S^0T) [+ coarse add]
#include <algorithm>

#include "fmp_common.h"

namespace fmp {
namespace {

constexpr int kLT = 256;      // threads
constexpr int kTI = 64;       // output rows per tile
constexpr int kTC = 64;       // output columns (pencils) per tile
constexpr int kKB = 16;       // k step

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

__device__ __forceinline__ bool box_wall(int q, int x, int y, int z) {
  return q == 0 ? (y == 0 || z == 0) : (q == 1 ? (x == 0 || z == 0) : (x == 0 || y == 0));
}

__device__ __forceinline__ long long buf_stride(const BoxDev& B) { return (3 * B.vol + 7) / 8 * 8; }

// Element (k, c) of a box component along `axis`: k the index along the
// axis, c the pencil (the other two indices, slower one first).
struct Walk {
  int sk, cdiv, sc1, sc2;
  // the pencil's part of the offset (a box component holds < 2^31 values);
  // element k of pencil c sits at k * sk + col(c)
  __device__ __forceinline__ int col(int c) const { return (c / cdiv) * sc1 + (c % cdiv) * sc2; }
};
__device__ __forceinline__ Walk walk_of(const BoxDev& B, int axis) {
  const int plane = B.nx * B.ny;
  if (axis == 0) return Walk{1, 1 << 30, 0, B.nx};          // c = (z, y): c * nx + k
  if (axis == 1) return Walk{B.nx, B.nx, plane, 1};         // c = (z, x)
  return Walk{plane, 1 << 30, 0, 1};                        // c = (y, x)
}

// ---------------------------------------------------------------- gather
// Work item (box, component, first plane of a slab of zs planes) -> copy 0.
template <typename T>
__global__ __launch_bounds__(kLT) void k_lg_gather(const double* __restrict__ r, T* __restrict__ W,
                                                   const BoxDev* __restrict__ boxes,
                                                   const DomainDev* __restrict__ doms,
                                                   const int4* __restrict__ work, int zs) {
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, plane = nx * ny;
  const int nzs = min(zs, B.nz - z0);
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  T* dst = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;
  for (int e = threadIdx.x; e < nzs * plane; e += kLT) {
    const int zl = e / plane, rem = e - zl * plane, y = rem / nx, x = rem - y * nx;
    const int z = z0 + zl;
    T v = T(0);
    if (!box_wall(q, x, y, z))
      v = (T)src[((long long)(B.bz0 + z) * D.ny + B.by0 + y) * D.nx + B.bx0 + x];
    dst[e] = v;
  }
}

// ---------------------------------------------------------------- contraction
// Even/odd butterfly of DCT-II / DST-I (the symmetry the vector-ALU passes
// use, here one level deep): along an axis of n with base tau (0 DCT-II,
// 1 DST-I), pairs (a_j, b_j) = (tau + j, n - 1 - j), j < P = (n - tau) / 2,
// and a middle index c when n - tau is odd (NS = P + mid).
//   forward:  out[tau + 2k]     = sum_j TS[k][j] (in[a_j] + in[b_j])   (k < NS; in[c] for j = P)
//             out[tau + 2k + 1] = sum_j TD[k][j] (in[a_j] - in[b_j])   (k < P)
//   inverse:  E_j = sum_k TS^T[j][k] y[tau + 2k],  O_j = sum_k TD^T[j][k] y[tau + 2k + 1]
//             x[a_j] = E_j + O_j, x[b_j] = E_j - O_j (j < P), x[c] = E_P
// (DST-I's slot 0 is the wall: zero).  Each is a GEMM over K = NS instead of
// n, so half the dense multiply-adds.  The tile rows are virtual rows:
// forward, rows [0, NSp) are the even outputs and [NSp, NSp + P) the odd
// ones (NSp = NS rounded up to 4, so a thread's four rows are of one kind);
// inverse, a thread's rows are E_j, E_j+1, O_j, O_j+1, so it combines its
// own pairs.  The input tile is staged twice per k step: the butterfly sums
// and differences (forward) or the even and odd coefficients (inverse).
struct HalfG {
  int tau, P, mid, NS, c;
};
__device__ __forceinline__ HalfG half_g(int n, int tau) {
  HalfG g;
  g.tau = tau;
  g.P = (n - tau) >> 1;
  g.mid = (n - tau) & 1;
  g.NS = g.P + g.mid;
  g.c = (n - 1 + tau) >> 1;
  return g;
}
__host__ __device__ __forceinline__ int round4(int v) { return (v + 3) & ~3; }

// Work item (box, component, row tile, column tile).  Copy `from` -> copy 1 - from.
template <typename T, bool inverse>
__global__ __launch_bounds__(kLT) void k_lg_contract(T* __restrict__ W,
                                                     const BoxDev* __restrict__ boxes,
                                                     const int4* __restrict__ work,
                                                     const T* __restrict__ tab, int axis,
                                                     int from) {
  __shared__ T As[kKB][kTI];
  __shared__ T Bs[kKB][kTC];                      // sums / even coefficients
  __shared__ T Bd[kKB][kTC];                      // differences / odd coefficients
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y;
  const int i0 = wk.z * kTI, c0 = wk.w * kTC;
  const int n = axis == 0 ? B.nx : (axis == 1 ? B.ny : B.nz);
  const int tau = q == axis ? 0 : 1;              // DCT-II along the own axis, DST-I else
  const HalfG g = half_g(n, tau);
  const int NSp = round4(g.NS);
  const int nrows = inverse ? 4 * ((g.NS + 1) >> 1) : NSp + g.P;
  if (i0 >= nrows) return;                        // the axis needs fewer row tiles
  const int ncol = (int)(B.vol / n);
  const Walk wlk = walk_of(B, axis);
  const long long bs = buf_stride(B);
  const T* src = W + B.w_off + (long long)from * bs + (long long)q * B.vol;
  T* dst = W + B.w_off + (long long)(1 - from) * bs + (long long)q * B.vol;
  // half tables TS, TD, TS^T, TD^T, hs x hs each: the side's own stride
  // (a large box can have sides of 48 cells or fewer on its other axes)
  const int hs = n <= kMaxSideVec ? kHS : kHL;
  const T* TS = tab + B.half[axis][tau];
  const T* TD = TS + hs * hs;
  const T* TSt = TS + 2 * hs * hs;
  const T* TDt = TS + 3 * hs * hs;
  const int t = threadIdx.x;
  const int ti = t >> 4, tj = t & 15;
  // table row of virtual row v, or null for a padding row
  auto arow = [&](int v) -> const T* {
    if constexpr (!inverse) {
      if (v < NSp) return v < g.NS ? TS + v * hs : nullptr;
      v -= NSp;
      return v < g.P ? TD + v * hs : nullptr;
    }
    const int j = 2 * (v >> 2) + (v & 1);
    if (j >= g.NS) return nullptr;
    return (v & 2) ? TDt + j * hs : TSt + j * hs;
  };
  // forward: a thread's four rows read the differences when they are odd
  // outputs; inverse: rows 0, 1 read the even coefficients, rows 2, 3 the odd
  const T (*Bf)[kTC] = (!inverse && i0 + ti * 4 >= NSp) ? Bd : Bs;
  // the thread's staging elements: (k in the step, pencil) fixed over the k
  // steps, so the pencil offsets are computed once (-1: beyond the pencils)
  constexpr int NJ = (kKB * kTC) / kLT;
  int sk_[NJ], sc_[NJ], scol[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int e = t + kLT * j;
    if (axis == 0) { sk_[j] = e % kKB; sc_[j] = e / kKB; }  // rows contiguous in memory
    else { sc_[j] = e % kTC; sk_[j] = e / kTC; }            // columns contiguous
    scol[j] = c0 + sc_[j] < ncol ? wlk.col(c0 + sc_[j]) : -1;
  }
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int k0 = 0; k0 < g.NS; k0 += kKB) {
#pragma unroll
    for (int j = 0; j < (kKB * kTI) / kLT; ++j) {   // table tile [k][virtual row]
      const int e = t + kLT * j, k = e % kKB, i = e / kKB;
      const T* row = arow(i0 + i);
      As[k][i] = (row && k0 + k < g.NS) ? row[k0 + k] : T(0);
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {                  // input tiles [k][c]
      const int kk = k0 + sk_[j];
      T sv = T(0), dv = T(0);
      if (scol[j] >= 0) {
        const T* col = src + scol[j];
        if constexpr (!inverse) {
          if (kk < g.P) {
            const T xa = col[(g.tau + kk) * wlk.sk], xb = col[(n - 1 - kk) * wlk.sk];
            sv = xa + xb;
            dv = xa - xb;
          } else if (kk == g.P && g.mid) {
            sv = col[g.c * wlk.sk];
          }
        } else {
          if (kk < g.NS) sv = col[(g.tau + 2 * kk) * wlk.sk];
          if (kk < g.P) dv = col[(g.tau + 2 * kk + 1) * wlk.sk];
        }
      }
      Bs[sk_[j]][sc_[j]] = sv;
      Bd[sk_[j]][sc_[j]] = dv;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKB; ++k) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[k][ti * 4 + a];
      if constexpr (inverse) {
        T bw[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          bv[b] = Bs[k][tj + 16 * b];
          bw[b] = Bd[k][tj + 16 * b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fmaT<T>(av[a], a < 2 ? bv[b] : bw[b], acc[a][b]);
      } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bf[k][tj + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fmaT<T>(av[a], bv[b], acc[a][b]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = c0 + tj + 16 * b;
    if (c >= ncol) continue;
    T* col = dst + wlk.col(c);
    const int sk = wlk.sk;
    if constexpr (!inverse) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int v = i0 + ti * 4 + a;
        int o = -1;
        if (v < NSp) { if (v < g.NS) o = g.tau + 2 * v; }
        else if (v - NSp < g.P) o = g.tau + 2 * (v - NSp) + 1;
        if (o >= 0) col[o * sk] = acc[a][b];
        if (v == 0 && g.tau) col[0] = T(0);         // DST-I: slot 0 holds no mode
      }
    } else {
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int j = 2 * ((i0 >> 2) + ti) + p;       // rows p (E_j) and p + 2 (O_j)
        if (j < g.P) {
          col[(g.tau + j) * sk] = acc[p][b] + acc[p + 2][b];
          col[(n - 1 - j) * sk] = acc[p][b] - acc[p + 2][b];
        } else if (j == g.P && g.mid) {
          col[g.c * sk] = acc[p][b];
        }
        if (j == 0 && g.tau) col[0] = T(0);         // DST-I: the wall slot
      }
    }
  }
}

// ---------------------------------------------------------------- solve
// Work item (box, component, slab) with component 0 only: the three
// components of every wavenumber (p, q, r) = (x, y, z) of the slab, in copy 1.
template <typename T>
__global__ __launch_bounds__(kLT) void k_lg_solve(T* __restrict__ W, const BoxDev* __restrict__ boxes,
                                                  const int4* __restrict__ work,
                                                  const T* __restrict__ tab, int zs) {
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  if (wk.y != 0) return;
  const BoxDev& B = boxes[wk.x];
  const int z0 = wk.z;
  const int nx = B.nx, ny = B.ny, plane = nx * ny;
  const int nzs = min(zs, B.nz - z0);
  T* w0 = W + B.w_off + buf_stride(B) + (long long)z0 * plane;
  const T* sx = tab + B.sig[0];
  const T* sy = tab + B.sig[1];
  const T* sz = tab + B.sig[2];
  const T alpha = (T)B.alpha;
  for (int e = threadIdx.x; e < nzs * plane; e += kLT) {
    const int zl = e / plane, rem = e - zl * plane, y = rem / nx, x = rem - y * nx;
    const T s1 = sx[x], s2 = sy[y], s3 = sz[z0 + zl];
    T* p0 = w0 + e;
    const T a = p0[0], b = p0[B.vol], d = p0[2 * B.vol];
    const T dot = fmaT<T>(s1, a, fmaT<T>(s2, b, s3 * d));
    const T den = fmaT<T>(alpha, fmaT<T>(s3, s3, fmaT<T>(s1, s1, s2 * s2)), T(1));
    const T inv = T(1) / den;
    p0[0] = fmaT<T>(alpha * s1, dot, a) * inv;
    p0[B.vol] = fmaT<T>(alpha * s2, dot, b) * inv;
    p0[2 * B.vol] = fmaT<T>(alpha * s3, dot, d) * inv;
  }
}

// ---------------------------------------------------------------- scatter
// Work item as the gather; copy 0 -> the owned unknowns of z (+ coarse).
template <typename T>
__global__ __launch_bounds__(kLT) void k_lg_scatter(const T* __restrict__ W, double* __restrict__ z,
                                                    const BoxDev* __restrict__ boxes,
                                                    const DomainDev* __restrict__ doms,
                                                    const int4* __restrict__ work, int zs,
                                                    const double* __restrict__ coarse, int nsub) {
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, plane = nx * ny;
  const int nzs = min(zs, B.nz - z0);
  const int lz0 = max(z0, B.oz0 - B.bz0), lz1 = min(z0 + nzs, B.oz0 - B.bz0 + B.sz);
  if (lz1 <= lz0) return;
  const int ly0 = B.oy0 - B.by0, lx0 = B.ox0 - B.bx0;
  const int oplane = B.sx * B.sy;
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const T* src = W + B.w_off + (long long)q * B.vol;
  const double cq = coarse ? coarse[(long long)q * nsub + B.sub] : 0.0;
  for (int e = threadIdx.x; e < (lz1 - lz0) * oplane; e += kLT) {
    const int zl = e / oplane, rem = e - zl * oplane, y = rem / B.sx, x = rem - y * B.sx;
    const int bz = lz0 + zl, by = ly0 + y, bx = lx0 + x;
    const int gx = B.bx0 + bx, gy = B.by0 + by, gz = B.bz0 + bz;
    double v = (double)src[(long long)bz * plane + by * nx + bx];
    if (coarse && !box_wall(q, gx, gy, gz)) v += cq;
    dst[((long long)gz * D.ny + gy) * D.nx + gx] = v;
  }
}

template <typename T>
hipError_t run_large(const double* r, void* Wv, double* z, const BoxDev* boxes,
                     const DomainDev* doms, const int4* work_a, int na, const int4* work_l,
                     const int* l0, const int* nl, int zs, const void* tabv, const double* coarse,
                     int nsub, hipStream_t s) {
  T* W = (T*)Wv;
  const T* tab = (const T*)tabv;
  hipLaunchKernelGGL((k_lg_gather<T>), dim3(na), dim3(kLT), 0, s, r, W, boxes, doms, work_a, zs);
  int from = 0;
  for (int a = 0; a < 3; ++a, from ^= 1)
    hipLaunchKernelGGL((k_lg_contract<T, false>), dim3(nl[a]), dim3(kLT), 0, s, W, boxes,
                       work_l + l0[a], tab, a, from);
  hipLaunchKernelGGL((k_lg_solve<T>), dim3(na), dim3(kLT), 0, s, W, boxes, work_a, tab, zs);
  for (int a = 2; a >= 0; --a, from ^= 1)
    hipLaunchKernelGGL((k_lg_contract<T, true>), dim3(nl[a]), dim3(kLT), 0, s, W, boxes,
                       work_l + l0[a], tab, a, from);
  hipLaunchKernelGGL((k_lg_scatter<T>), dim3(na), dim3(kLT), 0, s, W, z, boxes, doms, work_a, zs,
                     coarse, nsub);
  return hipGetLastError();
}

}  // namespace

int large_tile_rows() { return kTI; }
int large_rows(int n) {
  int r = n;
  for (int tau = 0; tau < 2; ++tau) {
    const int P = (n - tau) >> 1, NS = P + ((n - tau) & 1);
    r = std::max(r, std::max(round4(NS) + P, 4 * ((NS + 1) >> 1)));
  }
  return r;
}
int large_tile_cols() { return kTC; }

hipError_t launch_large(int prec, const double* r, void* W, double* z, const BoxDev* boxes,
                        const DomainDev* doms, const int4* work_a, int na, const int4* work_l,
                        const int* l0, const int* nl, int zs, const void* tab,
                        const double* coarse, int nsub, hipStream_t s) {
  if (na <= 0) return hipSuccess;
  if (prec == 0)
    return run_large<double>(r, W, z, boxes, doms, work_a, na, work_l, l0, nl, zs, tab, coarse,
                             nsub, s);
  return run_large<float>(r, W, z, boxes, doms, work_a, na, work_l, l0, nl, zs, tab, coarse, nsub,
                          s);
}

}  // namespace fmp
