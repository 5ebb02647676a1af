// FP64 vector kernels of the Krylov drivers (Sec. IV-A; Table III work per iteration).
//
// Reductions are two-stage with a fixed geometry: kRedBlocks blocks of 256
// threads each sum a fixed, strided subset of the elements, reduce inside the
// block in a fixed tree, and write one partial per block; a single block then
// sums the partials in a fixed order.  No atomics, so results are bitwise
// reproducible run to run.
//
// Scalars of BiCGSTAB live in a small device array S so that consecutive
// kernels consume them without a round trip to the host:
//   S[0] rho = <rhat, r>   S[1] rho_prev   S[2] alpha   S[3] omega
//   S[4] <rhat, v>         S[5] <t, s>     S[6] <t, t>  S[7] ||r||^2
//   S[8] beta
#include "fmp_common.h"

namespace fmp {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Reduce acc[0..n) over the block; thread 0 of each wave stores to lds, then
// threads i < n combine the 4 wave sums in order and write partials[i][blk].
template <int N>
__device__ __forceinline__ void block_store(const double (&acc)[N], int n, double* partials) {
  __shared__ double red[4][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i < n) {
      const double s = wave_sum(acc[i]);
      if (lane == 0) red[wave][i] = s;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < n) {
    const int i = threadIdx.x;
    partials[(long long)i * kRedBlocks + blockIdx.x] =
        ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
  }
}

__global__ __launch_bounds__(kThreads) void k_dots(DotPtrs P, int n, long long len,
                                                   double* __restrict__ partials) {
  double acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.0;
  const long long stride = (long long)kRedBlocks * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (i < n) acc[i] = __builtin_fma(P.a[i][e], P.b[i][e], acc[i]);
  }
  block_store<8>(acc, n, partials);
}

// Multi-vector kernels.  They are instantiated for the exact number of basis
// vectors (1..33): an unrolled loop guarded by a runtime count issues its
// loads in small groups and loses about a quarter of the bandwidth.
//
// Each block reads its segment (SegDev) and walks the segment's 16-byte pairs
// of doubles with the segment's block stride; thread 0 of the segment's first
// and last block take an odd leading and trailing element.  With one segment
// over the whole vector this is a plain grid-stride walk.
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <class P, class E>
__device__ __forceinline__ void seg_walk2(const SegDev& sg, P&& pair, E&& one) {
  const long long pa = (sg.e0 + 1) >> 1, pb = sg.e1 >> 1;
  const long long stride = (long long)sg.nb * kThreads;
  for (long long p = pa + (long long)((int)blockIdx.x - sg.b0) * kThreads + threadIdx.x; p < pb;
       p += stride)
    pair(p);
  if (threadIdx.x == 0) {
    if ((sg.e0 & 1) && (int)blockIdx.x == sg.b0) one(sg.e0);
    if ((sg.e1 & 1) && (int)blockIdx.x == sg.b0 + sg.nb - 1) one(sg.e1 - 1);
  }
}

// basis vectors are streamed once per pass: non-temporal loads
__device__ __forceinline__ dbl2 ld_stream(const double* __restrict__ base, long long p) {
  return __builtin_nontemporal_load(reinterpret_cast<const dbl2*>(base) + p);
}

template <int NV>
__global__ __launch_bounds__(kThreads) void k_mdot(const double* __restrict__ V, long long ldv,
                                                   const double* __restrict__ w,
                                                   const SegDev* __restrict__ map,
                                                   const int* __restrict__ act,
                                                   double* __restrict__ partials) {
  const SegDev sg = map[blockIdx.x];
  double acc[NV + 1];
#pragma unroll
  for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
  if (!act || act[sg.grp]) {
    const dbl2* __restrict__ w2 = reinterpret_cast<const dbl2*>(w);
    seg_walk2(
        sg,
        [&](long long p) {
          // all loads of the step are issued before the first product: the
          // compiler would otherwise consume each basis vector as it arrives
          // and keep only two or three loads in flight per wave
          dbl2 vv[NV];
#pragma unroll
          for (int i = 0; i < NV; ++i) vv[i] = ld_stream(V + i * ldv, p);
          const dbl2 we = w2[p];
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < NV; ++i)
            acc[i] = __builtin_fma(vv[i].x, we.x, __builtin_fma(vv[i].y, we.y, acc[i]));
          acc[NV] = __builtin_fma(we.x, we.x, __builtin_fma(we.y, we.y, acc[NV]));
        },
        [&](long long e) {
          const double we = w[e];
#pragma unroll
          for (int i = 0; i < NV; ++i) acc[i] = __builtin_fma(V[i * ldv + e], we, acc[i]);
          acc[NV] = __builtin_fma(we, we, acc[NV]);
        });
  }
  block_store<NV + 1>(acc, NV + 1, partials);   // <w,w> lands in column NV
}

// coefficients h_{g,i} * sc_{g,i} (sc = null: 1): the basis may be stored
// unnormalised, v_i = s_i * V_i, in which case sc_i = s_i^2
template <int NV>
__global__ __launch_bounds__(kThreads) void k_mupdate(const double* __restrict__ V, long long ldv,
                                                      const double* __restrict__ h,
                                                      const double* __restrict__ sc, int hld,
                                                      double* __restrict__ w,
                                                      const SegDev* __restrict__ map,
                                                      const int* __restrict__ act,
                                                      double* __restrict__ partials) {
  const SegDev sg = map[blockIdx.x];
  double acc[1] = {0.0};
  if (!act || act[sg.grp]) {
    double hh[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = h[sg.grp * hld + i] * (sc ? sc[sg.grp * hld + i] : 1.0);
    dbl2* __restrict__ w2 = reinterpret_cast<dbl2*>(w);
    seg_walk2(
        sg,
        [&](long long p) {
          dbl2 we = w2[p];
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            const dbl2 v = ld_stream(V + i * ldv, p);
            we.x = __builtin_fma(-hh[i], v.x, we.x);
            we.y = __builtin_fma(-hh[i], v.y, we.y);
          }
          w2[p] = we;
          acc[0] = __builtin_fma(we.x, we.x, __builtin_fma(we.y, we.y, acc[0]));
        },
        [&](long long e) {
          double we = w[e];
#pragma unroll
          for (int i = 0; i < NV; ++i) we = __builtin_fma(-hh[i], V[i * ldv + e], we);
          w[e] = we;
          acc[0] = __builtin_fma(we, we, acc[0]);
        });
  }
  block_store<1>(acc, 1, partials);
}

template <int NV>
__global__ __launch_bounds__(kThreads) void k_xupdate(const double* __restrict__ Z, long long ldz,
                                                      const double* __restrict__ y, int yld,
                                                      double* __restrict__ x,
                                                      const SegDev* __restrict__ map) {
  const SegDev sg = map[blockIdx.x];
  double yy[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) yy[i] = y[sg.grp * yld + i];
  dbl2* __restrict__ x2 = reinterpret_cast<dbl2*>(x);
  seg_walk2(
      sg,
      [&](long long p) {
        dbl2 xe = x2[p];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          const dbl2 v = ld_stream(Z + i * ldz, p);
          xe.x = __builtin_fma(yy[i], v.x, xe.x);
          xe.y = __builtin_fma(yy[i], v.y, xe.y);
        }
        x2[p] = xe;
      },
      [&](long long e) {
        double xe = x[e];
#pragma unroll
        for (int i = 0; i < NV; ++i) xe = __builtin_fma(yy[i], Z[i * ldz + e], xe);
        x[e] = xe;
      });
}

// same update for operands that are not 16-byte aligned
template <int NV>
__global__ __launch_bounds__(kThreads) void k_xupdate1(const double* __restrict__ Z, long long ldz,
                                                       int nz, const double* __restrict__ y,
                                                       int yld, double* __restrict__ x,
                                                       const SegDev* __restrict__ map) {
  const SegDev sg = map[blockIdx.x];
  double yy[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) yy[i] = (i < nz) ? y[sg.grp * yld + i] : 0.0;
  const long long stride = (long long)sg.nb * kThreads;
  for (long long e = sg.e0 + (long long)((int)blockIdx.x - sg.b0) * kThreads + threadIdx.x;
       e < sg.e1; e += stride) {
    double xe = x[e];
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i < nz) xe = __builtin_fma(yy[i], Z[i * ldz + e], xe);
    x[e] = xe;
  }
}

__global__ __launch_bounds__(kThreads) void k_scale_seg(const double* __restrict__ x,
                                                        const double* __restrict__ fac,
                                                        double* __restrict__ out,
                                                        const SegDev* __restrict__ map) {
  const SegDev sg = map[blockIdx.x];
  const double a = fac[sg.grp];
  if (a == 1.0 && x == out) return;   // in-place scaling by one: nothing to do
  const dbl2* __restrict__ x2 = reinterpret_cast<const dbl2*>(x);
  dbl2* __restrict__ o2 = reinterpret_cast<dbl2*>(out);
  seg_walk2(
      sg,
      [&](long long p) {
        const dbl2 v = x2[p];
        dbl2 r;
        r.x = a * v.x;
        r.y = a * v.y;
        o2[p] = r;
      },
      [&](long long e) { out[e] = a * x[e]; });
}

// Per-segment fixed-order reduction: thread t sums partial blocks b0 + t,
// b0 + t + 256, ... of its segment; waves and then the block combine in order.
// One workgroup per (segment, column): the columns, each summed in the same
// fixed order, go in parallel rather than one after another.
__global__ __launch_bounds__(kThreads) void k_reduce_seg(const double* __restrict__ partials,
                                                         const SegDev* __restrict__ segs,
                                                         double* __restrict__ out, int ostride) {
  __shared__ double red[4];
  const SegDev sg = segs[blockIdx.x];
  const int i = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const double* p = partials + (long long)i * kRedBlocks + sg.b0;
  double v = 0.0;
  for (int k = t; k < sg.nb; k += kThreads) v += p[k];
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (t == 0) out[(long long)blockIdx.x * ostride + i] = ((red[0] + red[1]) + red[2]) + red[3];
}

// post-op codes of the final reduction
enum { POST_NONE = 0, POST_ALPHA = 1, POST_OMEGA = 2, POST_RHO = 3 };

__global__ __launch_bounds__(kThreads) void k_reduce(const double* __restrict__ partials, int n,
                                                     double* __restrict__ out, int post,
                                                     double* __restrict__ S) {
  __shared__ double red[4];
  __shared__ double res[kMaxDots];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = 0; i < n; ++i) {
    const double* p = partials + (long long)i * kRedBlocks;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < kRedBlocks / kThreads; ++k) v += p[k * kThreads + t];
    v = wave_sum(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (t == 0) res[i] = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
  }
  if (t == 0) {
    for (int i = 0; i < n; ++i) out[i] = res[i];
    if (post == POST_ALPHA) {
      S[2] = S[0] / res[0];
    } else if (post == POST_OMEGA) {
      S[3] = res[1] > 0.0 ? res[0] / res[1] : 0.0;
    } else if (post == POST_RHO) {
      const double rho_new = res[1];
      S[8] = (rho_new / S[0]) * (S[2] / S[3]);
      S[1] = S[0];
      S[0] = rho_new;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_axpby(double a, const double* __restrict__ x,
                                                    double b, const double* __restrict__ y,
                                                    double* __restrict__ out, long long len) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride)
    out[e] = a * x[e] + b * y[e];
}

__global__ __launch_bounds__(kThreads) void k_scale_copy(const double* __restrict__ x, double a,
                                                         double* __restrict__ out, long long len) {
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride)
    out[e] = a * x[e];
}

// True 1 for a PEC-wall slot of a domain block: slot 0 along either node
// axis of the slot's component (x index i, y index j, z index k).
__device__ __forceinline__ bool wall_slot(const DomainDev& D, unsigned local) {
  const unsigned nxy = (unsigned)D.nx * (unsigned)D.ny;
  const unsigned cs = nxy * (unsigned)D.nz;
  const unsigned q = local / cs;
  const unsigned rem = local - q * cs;
  const unsigned k = rem / nxy;
  const unsigned rem2 = rem - k * nxy;
  const unsigned j = rem2 / (unsigned)D.nx;
  const unsigned i = rem2 - j * (unsigned)D.nx;
  return q == 0 ? (j == 0 || k == 0) : q == 1 ? (i == 0 || k == 0) : (i == 0 || j == 0);
}

__global__ __launch_bounds__(kThreads) void k_sub_norm(const double* __restrict__ b,
                                                       const double* __restrict__ y,
                                                       double* __restrict__ r,
                                                       const SegDev* __restrict__ map,
                                                       const DomainDev* __restrict__ doms,
                                                       double* __restrict__ partials) {
  const SegDev sg = map[blockIdx.x];
  const DomainDev D = doms[sg.dom];
  double acc[1] = {0.0};
  const long long stride = (long long)sg.nb * kThreads;
  for (long long e = sg.e0 + (long long)((int)blockIdx.x - sg.b0) * kThreads + threadIdx.x;
       e < sg.e1; e += stride) {
    const double v = wall_slot(D, (unsigned)(e - D.offset)) ? 0.0 : b[e] - y[e];
    r[e] = v;
    acc[0] = __builtin_fma(v, v, acc[0]);
  }
  block_store<1>(acc, 1, partials);
}

// blockIdx.y = 6 * domain + 2 * component + plane; plane 0 / 1 fixes the
// component's first / second node axis at 0
__global__ __launch_bounds__(kThreads) void k_zero_walls(double* __restrict__ x,
                                                         const DomainDev* __restrict__ doms) {
  const int d = blockIdx.y / 6, q = (blockIdx.y % 6) / 2, pl = blockIdx.y % 2;
  const DomainDev D = doms[d];
  const long long nxy = (long long)D.nx * D.ny, cs = nxy * D.nz;
  double* __restrict__ xq = x + D.offset + q * cs;
  // node axes: E_x (j, k), E_y (i, k), E_z (i, j); fix axis `fa` at 0
  const int fa = q == 0 ? (pl ? 2 : 1) : q == 1 ? (pl ? 2 : 0) : (pl ? 1 : 0);
  // the two free axes (a0 < a1): their extents and strides
  const int n0 = fa == 0 ? D.ny : D.nx;
  const int n1 = fa == 2 ? D.ny : D.nz;
  const long long s0 = fa == 0 ? (long long)D.nx : 1;
  const long long s1 = fa == 2 ? (long long)D.nx : nxy;
  const long long cnt = (long long)n0 * n1;
  for (long long t = (long long)blockIdx.x * kThreads + threadIdx.x; t < cnt;
       t += (long long)gridDim.x * kThreads) {
    const long long u = t % n0, v = t / n0;
    xq[u * s0 + v * s1] = 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void k_bicg_p(const double* __restrict__ r,
                                                     double* __restrict__ p,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ S, long long len) {
  const double beta = S[8], omega = S[3];
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride)
    p[e] = r[e] + beta * (p[e] - omega * v[e]);
}

__global__ __launch_bounds__(kThreads) void k_bicg_s(const double* __restrict__ r,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ sv,
                                                     const double* __restrict__ S, long long len) {
  const double alpha = S[2];
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride)
    sv[e] = r[e] - alpha * v[e];
}

__global__ __launch_bounds__(kThreads) void k_bicg_xr(double* __restrict__ x,
                                                      const double* __restrict__ phat,
                                                      const double* __restrict__ shat,
                                                      const double* __restrict__ sv,
                                                      const double* __restrict__ t,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ rhat,
                                                      const double* __restrict__ S, long long len,
                                                      double* __restrict__ partials) {
  const double alpha = S[2], omega = S[3];
  double acc[2] = {0.0, 0.0};
  const long long stride = (long long)kRedBlocks * kThreads;
  for (long long e = (long long)blockIdx.x * kThreads + threadIdx.x; e < len; e += stride) {
    x[e] = x[e] + alpha * phat[e] + omega * shat[e];
    const double re = sv[e] - omega * t[e];
    r[e] = re;
    acc[0] = __builtin_fma(re, re, acc[0]);
    acc[1] = __builtin_fma(rhat[e], re, acc[1]);
  }
  block_store<2>(acc, 2, partials);
}

int grid_for(long long len) {
  long long g = (len + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

// compile-time dispatch of a runtime basis count to its instantiation
template <int N>
struct NV {
  static void mdot(int nv, const double* V, long long ldv, const double* w, const SegDev* map,
                   const int* act, double* part, hipStream_t s) {
    if (nv == N)
      hipLaunchKernelGGL((k_mdot<N>), dim3(kRedBlocks), dim3(kThreads), 0, s, V, ldv, w, map, act,
                         part);
    else
      NV<N - 1>::mdot(nv, V, ldv, w, map, act, part, s);
  }
  static void mupdate(int nv, const double* V, long long ldv, const double* h, const double* sc,
                      int hld, double* w, const SegDev* map, const int* act, double* part,
                      hipStream_t s) {
    if (nv == N)
      hipLaunchKernelGGL((k_mupdate<N>), dim3(kRedBlocks), dim3(kThreads), 0, s, V, ldv, h, sc,
                         hld, w, map, act, part);
    else
      NV<N - 1>::mupdate(nv, V, ldv, h, sc, hld, w, map, act, part, s);
  }
  static void xupdate(int nz, const double* Z, long long ldz, const double* y, int yld, double* x,
                      const SegDev* map, hipStream_t s) {
    if (nz == N)
      hipLaunchKernelGGL((k_xupdate<N>), dim3(kRedBlocks), dim3(kThreads), 0, s, Z, ldz, y, yld, x,
                         map);
    else
      NV<N - 1>::xupdate(nz, Z, ldz, y, yld, x, map, s);
  }
};
template <>
struct NV<0> {
  static void mdot(int, const double*, long long, const double*, const SegDev*, const int*,
                   double*, hipStream_t) {}
  static void mupdate(int, const double*, long long, const double*, const double*, int, double*,
                      const SegDev*, const int*, double*, hipStream_t) {}
  static void xupdate(int, const double*, long long, const double*, int, double*, const SegDev*,
                      hipStream_t) {}
};

bool aligned16(const void* p) { return ((uintptr_t)p % 16) == 0; }

}  // namespace

hipError_t launch_dots(const DotPtrs& p, int n, long long len, double* partials, hipStream_t s) {
  if (n < 1 || n > 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks), dim3(kThreads), 0, s, p, n, len, partials);
  return hipGetLastError();
}

hipError_t launch_mdot(const double* V, long long ldv, int nv, const double* w,
                       const SegDev* map, const int* act, double* partials, hipStream_t s) {
  if (nv < 1 || nv + 1 > kMaxDots) return hipErrorInvalidValue;
  if (!aligned16(V) || !aligned16(w) || (ldv & 1)) return hipErrorInvalidValue;
  NV<33>::mdot(nv, V, ldv, w, map, act, partials, s);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int n, double* out, int post, double* S,
                         hipStream_t s) {
  if (n < 1 || n > kMaxDots) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, s, partials, n, out, post, S);
  return hipGetLastError();
}

hipError_t launch_reduce_seg(const double* partials, int n, const SegDev* segs, int nseg,
                             double* out, int ostride, hipStream_t s) {
  if (n < 1 || n > kMaxDots || nseg < 1 || nseg > kRedBlocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_seg, dim3(nseg, n), dim3(kThreads), 0, s, partials, segs, out,
                     ostride);
  return hipGetLastError();
}

hipError_t launch_mupdate(const double* V, long long ldv, int nv, const double* h,
                          const double* sc, int hld, double* w, const SegDev* map, const int* act,
                          double* partials, hipStream_t s) {
  if (nv < 1 || nv > 33) return hipErrorInvalidValue;
  if (!aligned16(V) || !aligned16(w) || (ldv & 1)) return hipErrorInvalidValue;
  NV<33>::mupdate(nv, V, ldv, h, sc, hld, w, map, act, partials, s);
  return hipGetLastError();
}

hipError_t launch_xupdate(const double* Z, long long ldz, int nz, const double* y, int yld,
                          double* x, const SegDev* map, hipStream_t s) {
  if (nz < 1 || nz > 33) return hipErrorInvalidValue;
  if (aligned16(Z) && aligned16(x) && (ldz % 2 == 0)) {
    NV<33>::xupdate(nz, Z, ldz, y, yld, x, map, s);
  } else {
#define L(NVV) \
  hipLaunchKernelGGL((k_xupdate1<NVV>), dim3(kRedBlocks), dim3(kThreads), 0, s, Z, ldz, nz, y, yld, x, map)
    if (nz <= 4) L(4);
    else if (nz <= 8) L(8);
    else if (nz <= 16) L(16);
    else L(33);
#undef L
  }
  return hipGetLastError();
}

hipError_t launch_scale_seg(const double* x, const double* fac, double* out, const SegDev* map,
                            hipStream_t s) {
  if (!aligned16(x) || !aligned16(out)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scale_seg, dim3(kRedBlocks), dim3(kThreads), 0, s, x, fac, out, map);
  return hipGetLastError();
}

hipError_t launch_zero_walls(double* x, const DomainDev* doms, int ndom, hipStream_t s) {
  if (ndom < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_walls, dim3(64, 6 * ndom), dim3(kThreads), 0, s, x, doms);
  return hipGetLastError();
}

hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out,
                        long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(len)), dim3(kThreads), 0, s, a, x, b, y, out, len);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double* x, double a, double* out, long long len,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(len)), dim3(kThreads), 0, s, x, a, out, len);
  return hipGetLastError();
}

hipError_t launch_sub_norm(const double* b, const double* y, double* r, const SegDev* map,
                           const DomainDev* doms, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_norm, dim3(kRedBlocks), dim3(kThreads), 0, s, b, y, r, map, doms,
                     partials);
  return hipGetLastError();
}

hipError_t launch_bicg_p(const double* r, double* p, const double* v, const double* S,
                         long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_p, dim3(grid_for(len)), dim3(kThreads), 0, s, r, p, v, S, len);
  return hipGetLastError();
}

hipError_t launch_bicg_s(const double* r, const double* v, double* sv, const double* S,
                         long long len, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_s, dim3(grid_for(len)), dim3(kThreads), 0, s, r, v, sv, S, len);
  return hipGetLastError();
}

hipError_t launch_bicg_xr(double* x, const double* phat, const double* shat, const double* sv,
                          const double* t, double* r, const double* rhat, const double* S,
                          long long len, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_xr, dim3(kRedBlocks), dim3(kThreads), 0, s, x, phat, shat, sv, t, r,
                     rhat, S, len, partials);
  return hipGetLastError();
}

}  // namespace fmp
