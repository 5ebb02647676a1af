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
#include <type_traits>

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

// One butterfly stage of the DCT-II / DST-I symmetry.  Both transforms pair
// the input index l with n-1-l: for DCT-II, T[p][n-1-l] = (-1)^p T[p][l]
// (pairs l = 0..P-1, base 0); for DST-I on slots 1..n-1, T[m][n-l] =
// (-1)^(m+1) T[m][l] (pairs l = 1..P, base 1).  With a_j = base + j,
// b_j = n-1-j, P = (n-base)/2 pairs and a middle index c = (n-1+base)/2 when
// n - base is odd:
//   sums  S_j = x[a_j] + x[b_j] (and S_P = x[c]) feed outputs base + 2k,
//   diffs D_j = x[a_j] - x[b_j]                 feed outputs base + 2k + 1,
// so a length-n transform is two half-size products.  The inverse (T^T) uses
// the same half tables transposed: E_j +- O_j give x[a_j] and x[b_j].
// Half tables per (side, type), each kHS x kHS, zero padded:
//   TS[k][j], TD[k][j] (forward rows), TS^T, TD^T (inverse rows).
struct Half {
  int n, base, P, mid, c;
};

__device__ __forceinline__ Half half_geom(int n, int tau) {
  Half g;
  g.n = n;
  g.base = tau;
  g.P = (n - tau) >> 1;
  g.mid = (n - tau) & 1;
  g.c = (n - 1 + tau) >> 1;
  return g;
}

// dot of a scalar-loaded table row with a register vector (two accumulators)
template <typename T, int NH>
__device__ __forceinline__ T row_dot(const T* __restrict__ row, const T (&v)[NH]) {
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int j = 0; j + 1 < NH; j += 2) {
    a0 = fmaT<T>(row[j], v[j], a0);
    a1 = fmaT<T>(row[j + 1], v[j + 1], a1);
  }
  if (NH & 1) a0 = fmaT<T>(row[NH - 1], v[NH - 1], a0);
  return a0 + a1;
}

// two rows at once: four independent FMA chains instead of two, with each
// output summed in the same order as row_dot (results are identical)
template <typename T, int NH>
__device__ __forceinline__ void row_dot2(const T* __restrict__ r0, const T* __restrict__ r1,
                                         const T (&v)[NH], T& o0, T& o1) {
  T a0 = T(0), a1 = T(0), b0 = T(0), b1 = T(0);
#pragma unroll
  for (int j = 0; j + 1 < NH; j += 2) {
    a0 = fmaT<T>(r0[j], v[j], a0);
    b0 = fmaT<T>(r1[j], v[j], b0);
    a1 = fmaT<T>(r0[j + 1], v[j + 1], a1);
    b1 = fmaT<T>(r1[j + 1], v[j + 1], b1);
  }
  if (NH & 1) {
    a0 = fmaT<T>(r0[NH - 1], v[NH - 1], a0);
    b0 = fmaT<T>(r1[NH - 1], v[NH - 1], b0);
  }
  o0 = a0 + a1;
  o1 = b0 + b1;
}

// one row of each of two tables times its own vector (the inverse's even and
// odd parts), four chains
template <typename T, int NH>
__device__ __forceinline__ void row_dot2(const T* __restrict__ r0, const T* __restrict__ r1,
                                         const T (&v0)[NH], const T (&v1)[NH], T& o0, T& o1) {
  T a0 = T(0), a1 = T(0), b0 = T(0), b1 = T(0);
#pragma unroll
  for (int j = 0; j + 1 < NH; j += 2) {
    a0 = fmaT<T>(r0[j], v0[j], a0);
    b0 = fmaT<T>(r1[j], v1[j], b0);
    a1 = fmaT<T>(r0[j + 1], v0[j + 1], a1);
    b1 = fmaT<T>(r1[j + 1], v1[j + 1], b1);
  }
  if (NH & 1) {
    a0 = fmaT<T>(r0[NH - 1], v0[NH - 1], a0);
    b0 = fmaT<T>(r1[NH - 1], v1[NH - 1], b0);
  }
  o0 = a0 + a1;
  o1 = b0 + b1;
}

// rows k0 .. k0+cnt-1 of a half table times v, two rows per step; the loop
// stays rolled so that two table rows at a time sit in SGPRs
template <typename T, int NH, class Out>
__device__ __forceinline__ void rows_times(const T* __restrict__ M, int cnt, const T (&v)[NH],
                                           Out out) {
#pragma unroll 1
  for (int k = 0; k + 1 < cnt; k += 2) {
    T o0, o1;
    row_dot2<T, NH>(M + k * kHS, M + (k + 1) * kHS, v, o0, o1);
    out(k, o0);
    out(k + 1, o1);
  }
  if (cnt & 1) out(cnt - 1, row_dot<T, NH>(M + (cnt - 1) * kHS, v));
}

// forward: y = T x; x read through ld(index), y written through st(index, value).
// TWO = false computes one output at a time (fewer registers: used where the
// caller already holds a whole pencil and register pressure sets occupancy).
template <typename T, int NH, bool TWO = true, class Load, class Store>
__device__ __forceinline__ void fwd_bfly(const T* __restrict__ tab, const Half g, Load ld,
                                         Store st) {
  T sv[NH], dv[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    T xa = T(0), xb = T(0);
    if (j < g.P) {
      xa = ld(g.base + j);
      xb = ld(g.n - 1 - j);
    } else if (j == g.P && g.mid) {
      xa = ld(g.c);
    }
    sv[j] = xa + xb;
    dv[j] = xa - xb;
  }
  const T* __restrict__ TS = tab;
  const T* __restrict__ TD = tab + kHS * kHS;
  const int NS = g.P + g.mid;
  if (TWO) {
    rows_times<T, NH>(TS, NS, sv, [&](int k, T val) { st(g.base + 2 * k, val); });
    rows_times<T, NH>(TD, g.P, dv, [&](int k, T val) { st(g.base + 2 * k + 1, val); });
  } else {
#pragma unroll 1
    for (int k = 0; k < NS; ++k) st(g.base + 2 * k, row_dot<T, NH>(TS + k * kHS, sv));
#pragma unroll 1
    for (int k = 0; k < g.P; ++k) st(g.base + 2 * k + 1, row_dot<T, NH>(TD + k * kHS, dv));
  }
  if (g.base) st(0, T(0));                        // DST-I: slot 0 holds no mode
}

// inverse: x = T^T y
template <typename T, int NH, bool TWO = true, class Load, class Store>
__device__ __forceinline__ void inv_bfly(const T* __restrict__ tab, const Half g, Load ld,
                                         Store st) {
  T ys[NH], yd[NH];
  const int NS = g.P + g.mid;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    ys[k] = (k < NS) ? ld(g.base + 2 * k) : T(0);
    yd[k] = (k < g.P) ? ld(g.base + 2 * k + 1) : T(0);
  }
  const T* __restrict__ TSt = tab + 2 * kHS * kHS;
  const T* __restrict__ TDt = tab + 3 * kHS * kHS;
#pragma unroll 1
  for (int j = 0; j < g.P; ++j) {                 // even and odd parts
    T e, o;
    if (TWO) {
      row_dot2<T, NH>(TSt + j * kHS, TDt + j * kHS, ys, yd, e, o);
    } else {
      e = row_dot<T, NH>(TSt + j * kHS, ys);
      o = row_dot<T, NH>(TDt + j * kHS, yd);
    }
    st(g.base + j, e + o);
    st(g.n - 1 - j, e - o);
  }
  if (g.mid) st(g.c, row_dot<T, NH>(TSt + g.P * kHS, ys));
  if (g.base) st(0, T(0));                        // DST-I: the wall slot
}

// Split forms for workgroups in which S = 2 or 4 threads share each pencil.
// The pencil is read in full by each of them (bfly_sums_or_diffs, inv_load),
// every thread of the workgroup passes a barrier, then each thread computes
// its share of the outputs: the forward splits by parity (even parts the
// sums' rows, i.e. the outputs base + 2k, odd parts the differences' rows)
// and, with four threads, each parity's rows in two halves; the inverse
// splits the output pairs j < P into S ranges (the last part also forms the
// middle index).  Every output is the same row product as in fwd_bfly /
// inv_bfly, summed in the same order, so the results are bitwise those of
// the unsplit forms.
template <typename T, int NH, class Load>
__device__ __forceinline__ void bfly_sums_or_diffs(const Half g, int part, Load ld, T (&u)[NH]) {
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    T xa = T(0), xb = T(0);
    if (j < g.P) {
      xa = ld(g.base + j);
      xb = ld(g.n - 1 - j);
    } else if (j == g.P && g.mid) {
      xa = ld(g.c);
    }
    u[j] = (part & 1) == 0 ? xa + xb : xa - xb;
  }
}

template <typename T, int NH, int S, class Store>
__device__ __forceinline__ void fwd_part(const T* __restrict__ tab, const Half g, int part,
                                         const T (&u)[NH], Store st) {
  const int odd = part & 1, piece = part >> 1;
  const int cnt = odd ? g.P : g.P + g.mid;
  const int step = (cnt + S / 2 - 1) / (S / 2);
  const int r0 = min(cnt, piece * step), r1 = min(cnt, r0 + step);
  const T* M = tab + (odd ? kHS * kHS : 0) + r0 * kHS;
  rows_times<T, NH>(M, r1 - r0, u, [&](int k, T val) { st(g.base + 2 * (r0 + k) + odd, val); });
  if (part == 0 && g.base) st(0, T(0));           // DST-I: slot 0 holds no mode
}

template <typename T, int NH, class Load>
__device__ __forceinline__ void inv_load(const Half g, Load ld, T (&ys)[NH], T (&yd)[NH]) {
  const int NS = g.P + g.mid;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    ys[k] = (k < NS) ? ld(g.base + 2 * k) : T(0);
    yd[k] = (k < g.P) ? ld(g.base + 2 * k + 1) : T(0);
  }
}

template <typename T, int NH, int S, class Store>
__device__ __forceinline__ void inv_part(const T* __restrict__ tab, const Half g, int part,
                                         const T (&ys)[NH], const T (&yd)[NH], Store st) {
  const T* __restrict__ TSt = tab + 2 * kHS * kHS;
  const T* __restrict__ TDt = tab + 3 * kHS * kHS;
  const int jm = (g.P + S - 1) / S;
  const int j0 = min(g.P, part * jm), j1 = min(g.P, j0 + jm);
#pragma unroll 1
  for (int j = j0; j < j1; ++j) {
    T e, o;
    row_dot2<T, NH>(TSt + j * kHS, TDt + j * kHS, ys, yd, e, o);
    st(g.base + j, e + o);
    st(g.n - 1 - j, e - o);
  }
  if (part == S - 1 && g.mid) st(g.c, row_dot<T, NH>(TSt + g.P * kHS, ys));
  if (part == 0 && g.base) st(0, T(0));           // DST-I: the wall slot
}

// 1/d for d >= 1 (the 3x3 solve's 1 + alpha |s|^2): a division in FP32; in
// FP64 the hardware estimate and one Newton step, which squares the
// estimate's relative error: the FP64 apply's error against the exact solve
// stays where it is with two steps (about 2e-15 relative on a 16^3 domain)
template <typename T>
__device__ __forceinline__ T recip(T d) {
  return T(1) / d;
}
template <>
__device__ __forceinline__ double recip<double>(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
}

// slot 0 of a component's node axes is the box wall
__device__ __forceinline__ bool box_wall(int q, int x, int y, int z) {
  return q == 0 ? (y == 0 || z == 0) : (q == 1 ? (x == 0 || z == 0) : (x == 0 || y == 0));
}


// Passes A and C work on slabs of kAC/NP planes (kAC pencils per direction):
// the FP64 slab then needs ~28 KB of LDS, 5 workgroups per CU.  The
// workgroups have 2 kAC threads, two per pencil (each forms half of the
// pencil's outputs), which doubles the waves per CU at the same LDS: at the
// 512 boxes of 34^3 of a 256^3 grid, FP64 pass A 347 -> 273 us and pass C
// 319 -> 274 us, FP32 pass A 216 -> 186 us.  FP32 pass C keeps one thread
// per pencil (its split form needs 104 VGPRs: 232 us against 177 us).  Four
// threads per pencil (512-thread workgroups) fit three FP64 workgroups per
// CU instead of five: pass A 334 us (FP32 224 us).
constexpr int kAC = 128;
template <int NP>
constexpr int zslab() {
  return kAC / NP;
}

// Slabs live in LDS densely as [zl][y][x] with the box's own strides, so a
// slab element's LDS index is its linear index e.  Loads of a thread are all
// issued before any is consumed (addresses clamped in bounds, results
// selected afterwards): the kernels are latency-bound otherwise.

// Calls f(n, tau) with the transform length n and the butterfly base tau as
// compile-time constants when n is NP or NP - 1 (the box sides of a class
// at the usual splits), so that the butterfly's index arithmetic folds into
// immediate offsets; other lengths take plain integers.  Used by pass A
// (FP64 at 256^3: 271 -> 252..262 us); in pass C the constant forms raise
// the register count from 85 to 151 (333 us), so it keeps the run-time form.
template <int NP, class F>
__device__ __forceinline__ void with_len(int n, int tau, F&& f) {
  using std::integral_constant;
  if (tau == 0) {
    if (n == NP) f(integral_constant<int, NP>{}, integral_constant<int, 0>{});
    else if (n == NP - 1) f(integral_constant<int, NP - 1>{}, integral_constant<int, 0>{});
    else f(n, 0);
  } else {
    if (n == NP) f(integral_constant<int, NP>{}, integral_constant<int, 1>{});
    else if (n == NP - 1) f(integral_constant<int, NP - 1>{}, integral_constant<int, 1>{});
    else f(n, 1);
  }
}

// ---------------------------------------------------------------- pass A
template <typename T, int NP, int NTH>
__global__ __launch_bounds__(NTH) void k_pass_a(const double* __restrict__ r, T* __restrict__ W,
                                                const BoxDev* __restrict__ boxes,
                                                const DomainDev* __restrict__ doms,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab) {
  static_assert(NTH == kAC || NTH == 2 * kAC || NTH == 4 * kAC, "1, 2 or 4 threads per pencil");
  constexpr int S = NTH / kAC;
  constexpr int ZS = zslab<NP>();
  constexpr int MAXE = (ZS * NP * NP + NTH - 1) / NTH;
  constexpr int NH = NP / 2;
  __shared__ T buf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const int plane = ny * nx;
  const int tot = nzs * plane;
  const int t = threadIdx.x;

  // S^gamma: gather the slab.  A thread's elements t + NTH i are stepped from
  // its first one by the fixed increment of NTH elements (two carries), with
  // no per-element division; loads of out-of-slab steps read element 0.
  // The box's wall slots (slot 0 of a node axis) are copied as they come:
  // the DST-I along that axis reads slots 1 .. n-1 only and writes zero to
  // its slot 0, and a wall row or plane feeds, through the transforms of the
  // other axes, only outputs at that same wall slot, which the DST-I along
  // the wall's own axis (here or in pass B) never reads.  So no value read
  // from a wall slot reaches a consumed coefficient.
  const double* s0 = src + ((long long)(B.bz0 + z0) * D.ny + B.by0) * D.nx + B.bx0;
  int zl = t / plane, y = (t - zl * plane) / nx, x = t - zl * plane - y * nx;
  const int dz = NTH / plane, rk = NTH - dz * plane, dy = rk / nx, dx = rk - dy * nx;
  int off = (zl * D.ny + y) * D.nx + x;
  const int doff = (dz * D.ny + dy) * D.nx + dx;
  const int cx_off = D.nx - nx, cy_off = (D.ny - ny) * D.nx;
  double vals[MAXE];
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {
    vals[i] = s0[t + NTH * i < tot ? off : 0];
    x += dx; y += dy; off += doff;
    if (x >= nx) { x -= nx; ++y; off += cx_off; }
    if (y >= ny) { y -= ny; off += cy_off; }
  }
#pragma unroll
  for (int i = 0; i < MAXE; ++i) {
    const int e = t + NTH * i;
    if (e < tot) buf[e] = (T)vals[i];
  }
  __syncthreads();

  const T* tabx = tab + B.half[0][q == 0 ? 0 : 1];
  const T* taby = tab + B.half[1][q == 1 ? 0 : 1];
  const Half gx = half_geom(nx, q == 0 ? 0 : 1), gy = half_geom(ny, q == 1 ? 0 : 1);
  T* dst0 = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;
  if constexpr (NTH == kAC) {
    if (t < nzs * ny) {                           // x, one row per lane (in place)
      T* row = buf + t * nx;
      fwd_bfly<T, NH>(tabx, gx, [&](int l) { return row[l]; }, [&](int p, T v) { row[p] = v; });
    }
    __syncthreads();
    if (t < nzs * nx) {                           // y, one column per lane, to the staging
      const int zl = t / nx, x = t - zl * nx;
      const T* colp = buf + zl * plane + x;
      T* dst = dst0 + zl * plane + x;
      fwd_bfly<T, NH>(taby, gy, [&](int m) { return colp[m * nx]; },
                      [&](int p, T v) { dst[p * nx] = v; });
    }
  } else {
    // S threads per pencil: waves 2p, 2p + 1 form part p of the outputs
    const int part = __builtin_amdgcn_readfirstlane(t / kAC);
    const int u = t - part * kAC;
    T hv[NH];
    T* row = buf + u * nx;
    with_len<NP>(nx, q == 0 ? 0 : 1, [&](auto n, auto tau) __attribute__((always_inline)) {
      const Half g = half_geom(n, tau);
      if (u < nzs * ny) bfly_sums_or_diffs<T, NH>(g, part, [&](int l) { return row[l]; }, hv);
      __syncthreads();                            // the row is overwritten in place
      if (u < nzs * ny) fwd_part<T, NH, S>(tabx, g, part, hv, [&](int p, T v) { row[p] = v; });
    });
    __syncthreads();
    if (u < nzs * nx) {
      const int zl = u / nx, x = u - zl * nx;
      const T* colp = buf + zl * plane + x;
      T* dst = dst0 + zl * plane + x;
      with_len<NP>(ny, q == 1 ? 0 : 1, [&](auto n, auto tau) __attribute__((always_inline)) {
        const Half g = half_geom(n, tau);
        bfly_sums_or_diffs<T, NH>(g, part, [&](int m) { return colp[m * nx]; }, hv);
        fwd_part<T, NH, S>(taby, g, part, hv, [&](int p, T v) { dst[p * nx] = v; });
      });
    }
  }
}

// ---------------------------------------------------------------- pass B
// Two forms.  The register-resident one (FP32) stages the whole spectral
// column set of a workgroup in LDS between the forward transform, the solve
// and the inverse, and computes two contraction rows at a time.  The ring
// form (FP64, further below) exchanges one wavenumber at a time: the FP64
// column set would need 52 KB of LDS per workgroup and cap occupancy there.

// The column is held in registers when its length nz is a compile-time
// constant (nz = NP or NP - 1, which covers every box of a class at the
// usual sides): the forward butterfly reads the registers and writes the
// spectral rows to LDS for the solve, and the inverse reads the solved rows
// back from registers.  Other lengths go through LDS.
template <typename T, int NP, int NZ, int TZ>
__device__ __forceinline__ void colz_fwd(const T* __restrict__ tabz, const T (&v)[NP],
                                         T (*exq)[64], int lane) {
  fwd_bfly<T, NP / 2, true>(tabz, half_geom(NZ, TZ), [&](int l) { return v[l]; },
                                     [&](int r, T val) { exq[r][lane] = val; });
}
template <typename T, int NP, int NZ, int TZ>
__device__ __forceinline__ void colz_inv(const T* __restrict__ tabz, const T (&e)[NP], T* col,
                                         int plane, bool active) {
  inv_bfly<T, NP / 2, true>(tabz, half_geom(NZ, TZ), [&](int r) { return e[r]; },
                                     [&](int l, T val) {
                                       if (active) col[(long long)l * plane] = val;
                                     });
}

template <typename T, int NP>
__global__ __launch_bounds__(192) void k_pass_b(T* __restrict__ W, const BoxDev* __restrict__ boxes,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab) {
  constexpr int NH = NP / 2;
  __shared__ T ex[3][NP][64];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  // one wave per component; readfirstlane tells the compiler q is wave-uniform,
  // so the table entries below stay scalar operands
  const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int plane = ny * nx;
  const int c = wk.y + lane;
  const bool active = c < plane;
  T* col = W + B.w_off + (long long)q * B.vol + (active ? c : 0);
  const int tz = q == 2 ? 0 : 1;                  // DCT-II along z for E_z, DST-I otherwise
  const T* tabz = tab + B.half[2][tz];
  // 0: nz = NP, 1: nz = NP - 1, 2: other (through LDS); uniform over the block
  const int form = nz == NP ? 0 : (nz == NP - 1 ? 1 : 2);

  T v[NP];                                        // the column, all loads in flight
#pragma unroll
  for (int l = 0; l < NP; ++l) v[l] = col[(long long)min(l, nz - 1) * plane];
  if (form == 0) {
    if (tz == 0) colz_fwd<T, NP, NP, 0>(tabz, v, ex[q], lane);
    else colz_fwd<T, NP, NP, 1>(tabz, v, ex[q], lane);
  } else if (form == 1) {
    if (tz == 0) colz_fwd<T, NP, NP - 1, 0>(tabz, v, ex[q], lane);
    else colz_fwd<T, NP, NP - 1, 1>(tabz, v, ex[q], lane);
  } else {
#pragma unroll
    for (int l = 0; l < NP; ++l) ex[q][l][lane] = v[l];
    const Half gz = half_geom(nz, tz);
    fwd_bfly<T, NH, true>(tabz, gz, [&](int l) { return ex[q][l][lane]; },
                                  [&](int r, T val) { ex[q][r][lane] = val; });
  }
  __syncthreads();

  // e = (r + alpha s (s.r)) / (1 + alpha |s|^2): wave q solves the wavenumbers
  // rr = q, q + 3, ... for all three components, in place
  const int yy = active ? c / nx : 0;
  const int xx = active ? c - yy * nx : 0;
  const T sx = tab[B.sig[0] + xx];
  const T sy = tab[B.sig[1] + yy];
  const T* sz = tab + B.sig[2];
  const T alpha = (T)B.alpha;
  const T sxy2 = fmaT<T>(sx, sx, sy * sy);
#pragma unroll
  for (int i = 0; i < (NP + 2) / 3; ++i) {
    const int rr = q + 3 * i;
    if (rr < NP) {
      const T s3 = sz[rr];
      const T a = ex[0][rr][lane], b = ex[1][rr][lane], d = ex[2][rr][lane];
      const T dot = fmaT<T>(sx, a, fmaT<T>(sy, b, s3 * d));
      const T inv = recip<T>(fmaT<T>(alpha, fmaT<T>(s3, s3, sxy2), T(1)));
      ex[0][rr][lane] = fmaT<T>(alpha * sx, dot, a) * inv;
      ex[1][rr][lane] = fmaT<T>(alpha * sy, dot, b) * inv;
      ex[2][rr][lane] = fmaT<T>(alpha * s3, dot, d) * inv;
    }
  }
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < NP; ++rr) v[rr] = ex[q][rr][lane];
  if (form == 0) {
    if (tz == 0) colz_inv<T, NP, NP, 0>(tabz, v, col, plane, active);
    else colz_inv<T, NP, NP, 1>(tabz, v, col, plane, active);
  } else if (form == 1) {
    if (tz == 0) colz_inv<T, NP, NP - 1, 0>(tabz, v, col, plane, active);
    else colz_inv<T, NP, NP - 1, 1>(tabz, v, col, plane, active);
  } else {
    inv_bfly<T, NH, true>(tabz, half_geom(nz, tz), [&](int r) { return ex[q][r][lane]; },
                                  [&](int l, T val) {
                                    if (active) col[(long long)l * plane] = val;
                                  });
  }
}

// Pass B, ring form.  The three waves (one per component) walk the z
// wavenumbers together, the even ones first, then the odd ones.  At each
// wavenumber a wave forms its component's forward coefficient (one half-table
// row times the butterfly sums or differences), the three coefficients meet
// in a two-slot LDS ring, every wave solves eq. (12) for its own component,
// and it adds the solved coefficient times the same table row into the
// inverse's even or odd accumulators (the inverse half tables are the
// transposes of the forward ones).  A table row is read once for both
// directions, and the LDS holds 2 x 3 x 64 values instead of the whole
// spectral column set.  Within one sweep a wave uses one butterfly half and
// one accumulator only: DCT-II takes its even modes from the sums and its odd
// modes from the differences, DST-I the reverse, so the first sweep runs
// over (sums, even accumulators) for E_z and (differences, odd accumulators)
// for E_x, E_y, and the second sweep over the other pair.  Three of the four
// half-length arrays are live at a time.
// FP64 only: with FP32 the register-resident form above is faster (135 us
// against 154 us or more for ring forms on the 512 boxes of 34^3 at 256^3),
// as its occupancy is not LDS-bound there.
template <typename T>
constexpr bool kPassBRing = sizeof(T) == 8;
template <typename T>
constexpr bool kRingPark = true;

template <typename T, int NP>
__global__ __launch_bounds__(192) void k_pass_b_ring(T* __restrict__ W,
                                                     const BoxDev* __restrict__ boxes,
                                                     const int4* __restrict__ work,
                                                     const T* __restrict__ tab) {
  constexpr int NH = NP / 2;
  static_assert(NP % 2 == 0, "size classes are even");
  __shared__ T ring[2][3][64];
  __shared__ T park[kRingPark<T> ? 3 : 1][kRingPark<T> ? NH : 1][64];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int plane = ny * nx;
  const int c = wk.y + lane;
  const bool active = c < plane;
  const int tz = q == 2 ? 0 : 1;                  // DCT-II along z for E_z, DST-I otherwise
  const T* __restrict__ TS = tab + B.half[2][tz];
  const T* __restrict__ TD = TS + kHS * kHS;
  const Half g = half_geom(nz, tz);
  const int NS = g.P + g.mid;

  // butterfly inputs: pair j is (base + j, n - 1 - j); every load is issued
  // (at a clamped, in-column index) before any is used.  u1 is the half the
  // first sweep uses (sums for DCT-II, differences for DST-I), u2 the other.
  // Addressed by 32-bit byte offsets from the component's (uniform) base:
  // one VGPR per load in flight (a box component is at most 96^3 values).
  T u1[NH], u2[NH];
  {
    const char* cb = reinterpret_cast<const char*>(W + B.w_off + (long long)q * B.vol);
    const unsigned c0 = (unsigned)(active ? c : 0);
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const unsigned la = (unsigned)min(g.base + j, nz - 1), lb = (unsigned)max(g.n - 1 - j, 0);
      u1[j] = *reinterpret_cast<const T*>(cb + (la * (unsigned)plane + c0) * (unsigned)sizeof(T));
      u2[j] = *reinterpret_cast<const T*>(cb + (lb * (unsigned)plane + c0) * (unsigned)sizeof(T));
    }
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    const T xa = u1[j], xb = u2[j];
    const T sum = j < g.P ? xa + xb : ((j == g.P && g.mid) ? xa : T(0));
    const T dif = j < g.P ? xa - xb : T(0);
    u1[j] = tz == 0 ? sum : dif;
    u2[j] = tz == 0 ? dif : sum;
  }
  const T* __restrict__ T1 = tz == 0 ? TS : TD;   // first sweep's half table
  const T* __restrict__ T2 = tz == 0 ? TD : TS;
  const int n1 = tz == 0 ? NS : g.P;              // rows of each
  const int n2 = tz == 0 ? g.P : NS;

  const int yy = active ? c / nx : 0;
  const int xx = active ? c - yy * nx : 0;
  const T sx = tab[B.sig[0] + xx];
  const T sy = tab[B.sig[1] + yy];
  const T* __restrict__ sz = tab + B.sig[2];
  const T alpha = (T)B.alpha;
  const T sxy2 = fmaT<T>(sx, sx, sy * sy);

  // the own component's solve at wavenumber rr from the three coefficients
  // in ring slot sl
  auto solve = [&](int rr, int sl) {
    const T a = ring[sl][0][lane], b = ring[sl][1][lane], d = ring[sl][2][lane];
    const T s3 = sz[rr];
    const T dot = fmaT<T>(sx, a, fmaT<T>(sy, b, s3 * d));
    const T inv = recip<T>(fmaT<T>(alpha, fmaT<T>(s3, s3, sxy2), T(1)));
    const T own = q == 0 ? a : (q == 1 ? b : d);
    const T sown = q == 0 ? sx : (q == 1 ? sy : s3);
    return fmaT<T>(alpha * sown, dot, own) * inv;
  };

  // the half not used by a sweep waits in LDS: u2 during the first sweep,
  // acc1 during the second, so that two half-length arrays are live in
  // registers at a time (more workgroups per CU)
  if constexpr (kRingPark<T>) {
#pragma unroll
    for (int j = 0; j < NH; ++j) park[q][j][lane] = u2[j];
  }
  T acc1[NH], acc2[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) acc1[j] = T(0);
  // step t = 0 .. NP-1 uses ring slot t & 1: even wavenumbers 2m first
  // (DCT-II row m of TS, DST-I row m - 1 of TD), then odd ones 2m + 1
  // (DCT-II row m of TD, DST-I row m of TS)
#pragma unroll 1
  for (int m = 0; m < NH; ++m) {
    const int k = m - tz;
    const bool has = k >= 0 && k < n1;
    const T* __restrict__ row = T1 + (has ? k : 0) * kHS;
    const T f = has ? row_dot<T, NH>(row, u1) : T(0);
    ring[m & 1][q][lane] = f;
    __syncthreads();
    const T e = solve(2 * m, m & 1);
    if (has) {
#pragma unroll
      for (int j = 0; j < NH; ++j) acc1[j] = fmaT<T>(row[j], e, acc1[j]);
    }
  }
  if constexpr (kRingPark<T>) {
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      u2[j] = park[q][j][lane];
      park[q][j][lane] = acc1[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) acc2[j] = T(0);
#pragma unroll 1
  for (int m = 0; m < NH; ++m) {
    const int t = NH + m;
    const bool has = m < n2;
    const T* __restrict__ row = T2 + (has ? m : 0) * kHS;
    const T f = has ? row_dot<T, NH>(row, u2) : T(0);
    ring[t & 1][q][lane] = f;
    __syncthreads();
    const T e = solve(2 * m + 1, t & 1);
    if (has) {
#pragma unroll
      for (int j = 0; j < NH; ++j) acc2[j] = fmaT<T>(row[j], e, acc2[j]);
    }
  }

  if constexpr (kRingPark<T>) {
#pragma unroll
    for (int j = 0; j < NH; ++j) acc1[j] = park[q][j][lane];
  }
  if (active) {
    // stores by 32-bit byte offsets from the component's base, as the loads
    char* cbw = reinterpret_cast<char*>(W + B.w_off + (long long)q * B.vol);
    const unsigned c0 = (unsigned)c;
    auto at = [&](int l) -> T& {
      return *reinterpret_cast<T*>(cbw + ((unsigned)l * (unsigned)plane + c0) * (unsigned)sizeof(T));
    };
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const T ev = tz == 0 ? acc1[j] : acc2[j];   // sums' (even) part
      const T od = tz == 0 ? acc2[j] : acc1[j];   // differences' (odd) part
      if (j < g.P) {
        at(g.base + j) = ev + od;
        at(g.n - 1 - j) = ev - od;
      } else if (j == g.P && g.mid) {
        at(g.c) = ev;
      }
    }
    if (g.base) at(0) = T(0);                     // DST-I: the wall slot
  }
}

// ---------------------------------------------------------------- pass C
template <typename T, int NP, int NTH>
__global__ __launch_bounds__(NTH) void k_pass_c(const T* __restrict__ W, double* __restrict__ z,
                                                const BoxDev* __restrict__ boxes,
                                                const DomainDev* __restrict__ doms,
                                                const int4* __restrict__ work,
                                                const T* __restrict__ tab,
                                                const double* __restrict__ coarse, int nsub) {
  static_assert(NTH == kAC || NTH == 2 * kAC || NTH == 4 * kAC, "1, 2 or 4 threads per pencil");
  constexpr int S = NTH / kAC;
  constexpr int ZS = zslab<NP>();
  constexpr int MAXE = (ZS * NP * NP + NTH - 1) / NTH;
  constexpr int NH = NP / 2;
  __shared__ T buf[ZS * NP * NP];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int plane = ny * nx;
  const int tot = nzs * plane;
  const int t = threadIdx.x;
  const int lz0 = max(z0, B.oz0 - B.bz0), lz1 = min(z0 + nzs, B.oz0 - B.bz0 + B.sz);
  if (lz1 <= lz0) return;                         // no owned plane in this slab
  const T* srcw = W + B.w_off + (long long)q * B.vol + (long long)z0 * plane;

  T vals[MAXE];                                   // the staged slab is contiguous
#pragma unroll
  for (int i = 0; i < MAXE; ++i) vals[i] = srcw[min(t + NTH * i, tot - 1)];
#pragma unroll
  for (int i = 0; i < MAXE; ++i)
    if (t + NTH * i < tot) buf[t + NTH * i] = vals[i];
  __syncthreads();

  const T* taby = tab + B.half[1][q == 1 ? 0 : 1];
  const T* tabx = tab + B.half[0][q == 0 ? 0 : 1];
  const Half gy = half_geom(ny, q == 1 ? 0 : 1), gx = half_geom(nx, q == 0 ? 0 : 1);
  if constexpr (NTH == kAC) {
    if (t < nzs * nx) {                           // y inverse, one column per lane (in place)
      const int zl = t / nx, x = t - zl * nx;
      T* colp = buf + zl * plane + x;
      inv_bfly<T, NH>(taby, gy, [&](int m) { return colp[m * nx]; },
                      [&](int m, T v) { colp[m * nx] = v; });
    }
    __syncthreads();
    if (t < nzs * ny) {                           // x inverse, one row per lane (in place)
      T* row = buf + t * nx;
      inv_bfly<T, NH>(tabx, gx, [&](int p) { return row[p]; }, [&](int l, T v) { row[l] = v; });
    }
  } else {
    // S threads per pencil: waves 2p, 2p + 1 form the outputs of the p-th
    // range of butterfly pairs; each pencil is read in full by all of them
    // before any overwrites it
    const int part = __builtin_amdgcn_readfirstlane(t / kAC);
    const int u = t - part * kAC;
    T ys[NH], yd[NH];
    {
      const int zl = u / nx, x = u - zl * nx;
      T* colp = buf + zl * plane + x;
      if (u < nzs * nx) inv_load<T, NH>(gy, [&](int m) { return colp[m * nx]; }, ys, yd);
      __syncthreads();
      if (u < nzs * nx)
        inv_part<T, NH, S>(taby, gy, part, ys, yd, [&](int m, T v) { colp[m * nx] = v; });
    }
    __syncthreads();
    T* row = buf + u * nx;
    if (u < nzs * ny) inv_load<T, NH>(gx, [&](int p) { return row[p]; }, ys, yd);
    __syncthreads();
    if (u < nzs * ny) inv_part<T, NH, S>(tabx, gx, part, ys, yd, [&](int l, T v) { row[l] = v; });
  }
  __syncthreads();

  // S^0T: write the owned part of the slab
  const int ly0 = B.oy0 - B.by0, lx0 = B.ox0 - B.bx0;
  const int oplane = B.sy * B.sx;
  const int otot = (lz1 - lz0) * oplane;
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const double cq = coarse ? coarse[(long long)q * nsub + B.sub] : 0.0;
  // owned element t + NTH i: (zl, y, x) stepped by the fixed increment of NTH
  // (two carries) with its slab index and its place in z
  const int sx = B.sx, sy = B.sy;
  int zl = t / oplane, y = (t - zl * oplane) / sx, x = t - zl * oplane - y * sx;
  const int dz = NTH / oplane, rk = NTH - dz * oplane, dy = rk / sx, dx = rk - dy * sx;
  int bi = (lz0 + zl - z0) * plane + (ly0 + y) * nx + lx0 + x;
  long long go = ((long long)(B.bz0 + lz0 + zl) * D.ny + (B.by0 + ly0 + y)) * D.nx + B.bx0 + lx0 + x;
  const int dbi = dz * plane + dy * nx + dx;
  const long long dgo = ((long long)dz * D.ny + dy) * D.nx + dx;
  const int cx_bi = nx - sx, cy_bi = plane - sy * nx;
  const long long cx_go = D.nx - sx, cy_go = (long long)(D.ny - sy) * D.nx;
  for (int e = t; e < otot; e += NTH) {
    double val = (double)buf[bi];
    if (coarse && !box_wall(q, B.bx0 + lx0 + x, B.by0 + ly0 + y, B.bz0 + lz0 + zl)) val += cq;
    dst[go] = val;
    x += dx; y += dy; zl += dz; bi += dbi; go += dgo;
    if (x >= sx) { x -= sx; ++y; bi += cx_bi; go += cx_go; }
    if (y >= sy) { y -= sy; ++zl; bi += cy_bi; go += cy_go; }
  }
}

// threads per workgroup of passes A and C: two per pencil, except in the
// FP32 pass C
template <typename T>
constexpr int kThreadsA = 2 * kAC;
template <typename T>
constexpr int kThreadsC = sizeof(T) == 8 ? 2 * kAC : kAC;

template <typename T, int NP>
hipError_t run_a(const double* r, void* W, const BoxDev* boxes, const DomainDev* doms,
                 const int4* work, int nwork, const void* tab, hipStream_t s) {
  constexpr int NTH = kThreadsA<T>;
  hipLaunchKernelGGL((k_pass_a<T, NP, NTH>), dim3(nwork), dim3(NTH), 0, s, r, (T*)W, boxes, doms,
                     work, (const T*)tab);
  return hipGetLastError();
}
template <typename T, int NP>
hipError_t run_b(void* W, const BoxDev* boxes, const int4* work, int nwork, const void* tab,
                 hipStream_t s) {
  if constexpr (kPassBRing<T>)
    hipLaunchKernelGGL((k_pass_b_ring<T, NP>), dim3(nwork), dim3(192), 0, s, (T*)W, boxes, work,
                       (const T*)tab);
  else
    hipLaunchKernelGGL((k_pass_b<T, NP>), dim3(nwork), dim3(192), 0, s, (T*)W, boxes, work,
                       (const T*)tab);
  return hipGetLastError();
}
template <typename T, int NP>
hipError_t run_c(const void* W, double* z, const BoxDev* boxes, const DomainDev* doms,
                 const int4* work, int nwork, const void* tab, const double* coarse, int nsub,
                 hipStream_t s) {
  constexpr int NTH = kThreadsC<T>;
  hipLaunchKernelGGL((k_pass_c<T, NP, NTH>), dim3(nwork), dim3(NTH), 0, s, (const T*)W, z, boxes,
                     doms, work, (const T*)tab, coarse, nsub);
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

int pass_a_zslab(int cls) { return kAC / kClasses[cls]; }

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
