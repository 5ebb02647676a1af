// Learned coarse correction on top of the RAS preconditioner, and the kernels
// that train it.
//
//   z = M_RAS^{-1} r + P0 ( ||R0 r|| * MLP( R0 r / ||R0 r|| ) )
//
// R0 averages r over the unknowns each subdomain owns, per component (a
// [3][nsub] coarse vector); P0 injects a coarse vector back as a constant per
// subdomain and component on the owned unknowns (fused into the last
// transform pass).  The MLP is in -> hidden (ReLU) -> hidden (ReLU) -> in with
// bf16 weights and FP32 accumulation.  Dividing by ||R0 r|| and multiplying
// back makes the correction scale with r like a linear preconditioner.
//
// The FP64 residual decides on the correction inside FGMRES: with v the
// preconditioner input, z = z_RAS + d and w = A z, the kernel k_resid_test
// compares ||v - w|| (with the correction) against ||v - w + A d|| (plain
// RAS) in one pass over v and w, evaluating A d = d + c/eps K d on the fly
// from the piecewise-constant d (K d vanishes inside a subdomain).  When the
// correction does not reduce the residual the solver falls back to the plain
// preconditioner for that step.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "fmp_common.h"
#include "fmp_ctx.h"

using namespace fmp;

// Device scratch of fmp_mlp_loss_grad_noalloc: one copy per GPU, alive until
// the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host it is a stand-in, not a device address): it takes the device
// address hipGetSymbolAddress returns for the current GPU, once per GPU.
static constexpr size_t kMlpStaticScratchBytes = FMP_MLP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kMlpStaticScratchBytes];

namespace {

constexpr int kHidMax = 512;
constexpr int kT = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// fixed-order block sum of one double (result valid in thread 0)
__device__ __forceinline__ double block_sum_d(double v, double* red4) {
  v = wave_sum_d(v);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = ((red4[0] + red4[1]) + red4[2]) + red4[3];
  __syncthreads();
  return s;
}

__device__ __forceinline__ bool is_wall(int q, int i, int j, int k) {
  return q == 0 ? (j == 0 || k == 0) : (q == 1 ? (i == 0 || k == 0) : (i == 0 || j == 0));
}

// ---------------------------------------------------------------- R0
// one block per (subdomain, component): mean over the owned unknowns
__global__ __launch_bounds__(kT) void k_restrict(const double* __restrict__ r,
                                                 const BoxDev* __restrict__ boxes,
                                                 const DomainDev* __restrict__ doms, int nsub,
                                                 double* __restrict__ rc) {
  __shared__ double red[4];
  const int s = blockIdx.x, q = blockIdx.y;
  const BoxDev& B = boxes[s];
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const int n = B.sx * B.sy * B.sz;
  double acc = 0.0, cnt = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) {
    const int z = e / (B.sx * B.sy), rem = e - z * B.sx * B.sy, y = rem / B.sx, x = rem - y * B.sx;
    const int gi = B.ox0 + x, gj = B.oy0 + y, gk = B.oz0 + z;
    if (!is_wall(q, gi, gj, gk)) {
      acc += src[((long long)gk * D.ny + gj) * D.nx + gi];
      cnt += 1.0;
    }
  }
  const double sum = block_sum_d(acc, red);
  const double num = block_sum_d(cnt, red);
  if (threadIdx.x == 0) rc[(long long)q * nsub + s] = num > 0.0 ? sum / num : 0.0;
}

// ---------------------------------------------------------------- MLP inference
// u = rc / ||rc|| (FP32), S[0] = ||rc||
__global__ __launch_bounds__(kT) void k_coarse_in(const double* __restrict__ rc, int n,
                                                  float* __restrict__ u, double* __restrict__ S) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int e = threadIdx.x; e < n; e += kT) acc = __builtin_fma(rc[e], rc[e], acc);
  const double nrm = sqrt(block_sum_d(acc, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int e = threadIdx.x; e < n; e += kT) u[e] = (float)(rc[e] * inv);
  if (threadIdx.x == 0) S[0] = nrm;
}

// y[row] = act(W[row] . x + b[row]); one wave per row, W bf16 row-major
__global__ __launch_bounds__(kT) void k_gemv(const __hip_bfloat16* __restrict__ W,
                                             const float* __restrict__ b,
                                             const float* __restrict__ x, int rows, int cols,
                                             int relu, float* __restrict__ y,
                                             double* __restrict__ yd,
                                             const double* __restrict__ S) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  const __hip_bfloat16* w = W + (long long)row * cols;
  float acc = 0.f;
  for (int c = lane; c < cols; c += 64) acc = __builtin_fmaf(__bfloat162float(w[c]), x[c], acc);
  acc = wave_sum_f(acc);
  if (lane == 0) {
    float v = acc + b[row];
    if (relu) v = v > 0.f ? v : 0.f;
    if (yd) yd[row] = S[0] * (double)v;   // last layer: scale back by ||R0 r||
    else y[row] = v;
  }
}

// ---------------------------------------------------------------- residual test
// d(q, k, j, i): the piecewise-constant correction on unknown slots
// v / d for 0 <= v < 2^20 from a precomputed float 1/d: the rounding error of
// (v + 1/2) / d in FP32 stays far below its 1/(2d) margin to the next integer
__device__ __forceinline__ int fquot(int v, float inv_d) { return (int)(((float)v + 0.5f) * inv_d); }

// The field is evaluated around one centre slot (i0, j0, k0) at a time: the
// centre's subdomain coordinates (si, sj, sk) and its position inside that
// subdomain (li, lj, lk) are computed once, and a neighbour one cell away
// lies in the same subdomain or the next one along that axis (subdomains
// have equal sides within a domain).
struct CoarseField {
  const double* yc;
  int nsub;
  DomainDev D;
  int i0, j0, k0;
  int si, sj, sk, li, lj, lk;
  // branch-free, so that the loads of all stencil terms are issued together:
  // a slot outside the domain or on a wall reads a clamped in-range entry
  // and yields 0
  __device__ __forceinline__ double operator()(int q, int k, int j, int i) const {
    const bool ok = i >= 0 && j >= 0 && k >= 0 && i < D.nx && j < D.ny && k < D.nz &&
                    !is_wall(q, i, j, k);
    const int ai = li + (i - i0), aj = lj + (j - j0), ak = lk + (k - k0);
    const int ti = min(max(si + (ai < 0 ? -1 : (ai >= D.sx ? 1 : 0)), 0), D.px - 1);
    const int tj = min(max(sj + (aj < 0 ? -1 : (aj >= D.sy ? 1 : 0)), 0), D.py - 1);
    const int tk = min(max(sk + (ak < 0 ? -1 : (ak >= D.sz ? 1 : 0)), 0), D.pz - 1);
    const double v = yc[(long long)q * nsub + D.sub0 + (tk * D.py + tj) * D.px + ti];
    return ok ? v : 0.0;
  }
};

// cell permittivity; the block index comes from a reciprocal of the block
// side (coordinates are non-negative and below 2^20)
__device__ __forceinline__ double cell_eps(const double* __restrict__ e, const DomainDev& D,
                                           float inv_b, int i, int j, int k) {
  return e[D.eps_off + (fquot(k, inv_b) * D.eps_nby + fquot(j, inv_b)) * D.eps_nbx +
           fquot(i, inv_b)];
}

// (A d) at slot (q, k, j, i), the same 13-point double-curl as the stencil
// kernel.  Away from subdomain faces and the walls K d = 0 exactly, so the
// slot's own value is returned; the face slots of a wave (a few lanes of each
// 64-slot row) take the full stencil, whose neighbour lookups are cheap.
__device__ double apply_A_at(const CoarseField& d, const DomainDev& D,
                             const double* __restrict__ eps, float inv_b, int q, int k, int j,
                             int i) {
  if (is_wall(q, i, j, k)) return 0.0;
  const double c0 = d(q, k, j, i);
  if (d.li >= 1 && d.li + 1 < D.sx && d.lj >= 1 && d.lj + 1 < D.sy && d.lk >= 1 &&
      d.lk + 1 < D.sz && i >= 2 && j >= 2 && k >= 2 && i + 2 < D.nx && j + 2 < D.ny &&
      k + 2 < D.nz)
    return c0;
  double kd, sc = D.c;
  if (q == 0) {
    kd = 4.0 * c0 - d(0, k, j + 1, i) - d(0, k, j - 1, i) - d(0, k + 1, j, i) - d(0, k - 1, j, i) +
         (d(1, k, j, i + 1) - d(1, k, j, i) - d(1, k, j - 1, i + 1) + d(1, k, j - 1, i)) +
         (d(2, k, j, i + 1) - d(2, k, j, i) - d(2, k - 1, j, i + 1) + d(2, k - 1, j, i));
    if (D.eps_b > 0)
      sc = D.c / (0.25 * (((cell_eps(eps, D, inv_b, i, j - 1, k - 1) +
                            cell_eps(eps, D, inv_b, i, j - 1, k)) +
                           cell_eps(eps, D, inv_b, i, j, k - 1)) +
                          cell_eps(eps, D, inv_b, i, j, k)));
  } else if (q == 1) {
    kd = 4.0 * c0 - d(1, k + 1, j, i) - d(1, k - 1, j, i) - d(1, k, j, i + 1) - d(1, k, j, i - 1) +
         (d(2, k, j + 1, i) - d(2, k, j, i) - d(2, k - 1, j + 1, i) + d(2, k - 1, j, i)) +
         (d(0, k, j + 1, i) - d(0, k, j, i) - d(0, k, j + 1, i - 1) + d(0, k, j, i - 1));
    if (D.eps_b > 0)
      sc = D.c / (0.25 * (((cell_eps(eps, D, inv_b, i - 1, j, k - 1) +
                            cell_eps(eps, D, inv_b, i - 1, j, k)) +
                           cell_eps(eps, D, inv_b, i, j, k - 1)) +
                          cell_eps(eps, D, inv_b, i, j, k)));
  } else {
    kd = 4.0 * c0 - d(2, k, j, i + 1) - d(2, k, j, i - 1) - d(2, k, j + 1, i) - d(2, k, j - 1, i) +
         (d(0, k + 1, j, i) - d(0, k, j, i) - d(0, k + 1, j, i - 1) + d(0, k, j, i - 1)) +
         (d(1, k + 1, j, i) - d(1, k, j, i) - d(1, k + 1, j - 1, i) + d(1, k, j - 1, i));
    if (D.eps_b > 0)
      sc = D.c / (0.25 * (((cell_eps(eps, D, inv_b, i - 1, j - 1, k) +
                            cell_eps(eps, D, inv_b, i - 1, j, k)) +
                           cell_eps(eps, D, inv_b, i, j - 1, k)) +
                          cell_eps(eps, D, inv_b, i, j, k)));
  }
  return c0 + sc * kd;
}

// partials: [0] ||v - w||^2 (with the correction), [1] ||v - w + A d||^2 (plain)
__global__ __launch_bounds__(kT) void k_resid_test(const double* __restrict__ v,
                                              const double* __restrict__ w,
                                              const double* __restrict__ yc, int nsub,
                                              const DomainDev* __restrict__ doms, int ndom,
                                              const double* __restrict__ eps, long long len,
                                              double* __restrict__ partials) {
  __shared__ double red[4][2];
  double a0 = 0.0, a1 = 0.0;
  const long long stride = (long long)kRedBlocks * kT;
  // the element -> (q, k, j, i) decomposition uses quotients from reciprocals
  // computed once per domain (exact: FP64 for offsets within a vector and a
  // plane, FP32 for single coordinates, which stay below 2^20)
  int d = -1;
  DomainDev D{};
  long long cs = 1;
  int pl = 1;
  double inv_cs = 1.0, inv_pl = 1.0;
  double inv_nx = 1.0;
  float inv_sx = 1.f, inv_sy = 1.f, inv_sz = 1.f, inv_b = 1.f;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < len; e += stride) {
    int dn = d < 0 ? 0 : d;
    while (dn + 1 < ndom && e >= doms[dn + 1].offset) ++dn;
    if (dn != d) {
      d = dn;
      D = doms[d];
      pl = D.ny * D.nx;
      cs = (long long)D.nz * pl;
      inv_cs = 1.0 / (double)cs;
      inv_pl = 1.0 / (double)pl;
      inv_nx = 1.0 / (double)D.nx;
      inv_sx = 1.f / (float)D.sx;
      inv_sy = 1.f / (float)D.sy;
      inv_sz = 1.f / (float)D.sz;
      inv_b = D.eps_b > 0 ? 1.f / (float)D.eps_b : 1.f;
    }
    const long long loc = e - D.offset;
    const int q = (int)(((double)loc + 0.5) * inv_cs);
    const long long rem = loc - q * cs;
    const int k = (int)(((double)rem + 0.5) * inv_pl);
    const int rr = (int)(rem - (long long)k * pl);
    const int j = (int)(((double)rr + 0.5) * inv_nx), i = rr - j * D.nx;
    const int si = fquot(i, inv_sx), sj = fquot(j, inv_sy), sk = fquot(k, inv_sz);
    const CoarseField F{yc, nsub, D, i, j, k, si, sj, sk,
                        i - si * D.sx, j - sj * D.sy, k - sk * D.sz};
    const double ad = apply_A_at(F, D, eps, inv_b, q, k, j, i);
    const double rl = v[e] - w[e];
    const double rp = rl + ad;
    a0 = __builtin_fma(rl, rl, a0);
    a1 = __builtin_fma(rp, rp, a1);
  }
  a0 = wave_sum_d(a0);
  a1 = wave_sum_d(a1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { red[wave][0] = a0; red[wave][1] = a1; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int i = threadIdx.x;
    partials[(long long)i * kRedBlocks + blockIdx.x] =
        ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
  }
}

// ---------------------------------------------------------------- training GEMM
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  const float* A; long long sam, sak;     // A(m, k)
  const float* B; long long sbk, sbn;     // B(k, n)
  float* C; long long scm, scn;           // C(m, n)
  int M, N, K;
  const float* bias;                      // + bias[n]
  int relu;                               // max(., 0)
  const float* mask; long long smm, smn;  // * (mask(m, n) > 0)
};

// C = A B on the matrix cores: 64 x 64 tile per block, K in steps of 32,
// operands rounded to bf16 when staged in LDS, FP32 accumulation.
__global__ __launch_bounds__(kT) void k_gemm(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[64][40];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[64][40];   // Bs[n][k]
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  f32x4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int lr = t >> 2, lk = (t & 3) * 8;
  for (int k0 = 0; k0 < g.K; k0 += 32) {
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int m = m0 + lr, n = n0 + lr, k = k0 + lk + jj;
      As[lr][lk + jj] = (__bf16)((m < g.M && k < g.K) ? g.A[m * g.sam + k * g.sak] : 0.f);
      Bs[lr][lk + jj] = (__bf16)((n < g.N && k < g.K) ? g.B[k * g.sbk + n * g.sbn] : 0.f);
    }
    __syncthreads();
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wave * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[nt * 16 + (lane & 15)][8 * (lane >> 4)]);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nt], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + wave * 16 + 4 * (lane >> 4) + i, n = n0 + nt * 16 + (lane & 15);
      if (m < g.M && n < g.N) {
        float v = acc[nt][i];
        if (g.bias) v += g.bias[n];
        if (g.relu) v = v > 0.f ? v : 0.f;
        if (g.mask) v = g.mask[m * g.smm + n * g.smn] > 0.f ? v : 0.f;
        g.C[m * g.scm + n * g.scn] = v;
      }
    }
}

hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm, dim3((g.N + 63) / 64, (g.M + 63) / 64), dim3(kT), 0, s, g);
  return hipGetLastError();
}

// dO = 2 (O - Y) / (rows*cols); per-block partial sums of (O - Y)^2
__global__ __launch_bounds__(kT) void k_mse(const float* __restrict__ O, const float* __restrict__ Y,
                                            long long n, float scale, float* __restrict__ dO,
                                            double* __restrict__ partials) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * kT + threadIdx.x; e < n; e += (long long)gridDim.x * kT) {
    const float d = O[e] - Y[e];
    dO[e] = 2.f * d * scale;
    acc += (double)d * (double)d;
  }
  const double s = block_sum_d(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_mse_final(const double* __restrict__ partials, int nb, double scale,
                            float* __restrict__ loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += partials[i];
    *loss = (float)(s * scale);
  }
}

// db[n] = sum_m dZ[m][n], rows summed in order
__global__ __launch_bounds__(kT) void k_colsum(const float* __restrict__ dZ, int M, int N,
                                               float* __restrict__ db) {
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(long long)m * N + n];
  db[n] = s;
}

__global__ __launch_bounds__(kT) void k_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v,
                                             float lr, float bc1, float bc2) {
  const int i = blockIdx.x * kT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

uint16_t to_bf16_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

}  // namespace

// ============================================================== host side
size_t fmp_coarse_workspace(int nsub, int hidden_max) {
  const size_t in = 3 * (size_t)nsub, H = hidden_max;
  return al(in * 8) * 2 + al(64) + al(in * 4) + al(H * 4) * 2 + al(H * in * 2) * 2 +
         al(H * H * 2) + al(H * 4) * 2 + al(in * 4);
}

void fmp_coarse_bind(fmp_ctx* h, void* base) {
  const size_t in = 3 * (size_t)h->nsub, H = kHidMax;
  char* p = (char*)base;
  auto take = [&](size_t bytes) { char* r = p; p += al(bytes); return r; };
  h->d_rc = (double*)take(in * 8);
  h->d_yc = (double*)take(in * 8);
  h->d_cS = (double*)take(64);
  h->d_u = (float*)take(in * 4);
  h->d_h1 = (float*)take(H * 4);
  h->d_h2 = (float*)take(H * 4);
  h->d_W1 = (__hip_bfloat16*)take(H * in * 2);
  h->d_W3 = (__hip_bfloat16*)take(H * in * 2);
  h->d_W2 = (__hip_bfloat16*)take(H * H * 2);
  h->d_b1 = (float*)take(H * 4);
  h->d_b2 = (float*)take(H * 4);
  h->d_b3 = (float*)take(in * 4);
}

static hipError_t restrict_launch(fmp_ctx* h, const double* r, double* rc, hipStream_t s) {
  if (h->nsub <= 0 || h->boxes.empty()) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_restrict, dim3(h->nsub, 3), dim3(kT), 0, s, r, h->d_boxes, h->d_doms,
                     h->nsub, rc);
  return hipGetLastError();
}

// R0 r -> MLP -> h->d_yc (the correction to inject); *out = d_yc
fmp_status fmp_coarse_forward(fmp_ctx* h, const double* r, hipStream_t s, const double** out) {
  *out = nullptr;
  if (!h->learned_set) return FMP_OK;
  const int in = 3 * h->nsub, H = h->hidden;
  hipError_t e = restrict_launch(h, r, h->d_rc, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_coarse_in, dim3(1), dim3(kT), 0, s, h->d_rc, in, h->d_u, h->d_cS);
    hipLaunchKernelGGL(k_gemv, dim3((H + 3) / 4), dim3(kT), 0, s, h->d_W1, h->d_b1, h->d_u, H, in,
                       1, h->d_h1, (double*)nullptr, (const double*)nullptr);
    hipLaunchKernelGGL(k_gemv, dim3((H + 3) / 4), dim3(kT), 0, s, h->d_W2, h->d_b2, h->d_h1, H, H,
                       1, h->d_h2, (double*)nullptr, (const double*)nullptr);
    hipLaunchKernelGGL(k_gemv, dim3((in + 3) / 4), dim3(kT), 0, s, h->d_W3, h->d_b3, h->d_h2, in,
                       H, 0, (float*)nullptr, h->d_yc, (const double*)h->d_cS);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    h->err = std::string("coarse forward: ") + hipGetErrorString(e);
    return FMP_ERR_HIP;
  }
  *out = h->d_yc;
  return FMP_OK;
}

// one pass over v, w: partials of ||v - w||^2 and ||v - w + A d||^2
hipError_t fmp_coarse_resid_test(fmp_ctx* h, const double* v, const double* w, double* partials,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_resid_test, dim3(kRedBlocks), dim3(kT), 0, s, v, w, (const double*)h->d_yc,
                     h->nsub, h->d_doms, (int)h->doms.size(), h->d_eps, h->len, partials);
  return hipGetLastError();
}

extern "C" {

fmp_status fmp_coarse_size(fmp_handle h, int32_t* n) {
  if (!h || !n) return FMP_ERR_INVALID_ARG;
  *n = 3 * h->nsub;
  return FMP_OK;
}

fmp_status fmp_set_coarse_model(fmp_handle h, int32_t hidden, const float* w, size_t bytes) {
  if (!h) return FMP_ERR_INVALID_ARG;
  if (!h->use_learned || !h->precond_ok) return FMP_ERR_UNSUPPORTED;
  if (!w) {
    h->learned_set = false;
    return FMP_OK;
  }
  const size_t in = 3 * (size_t)h->nsub;
  if (hidden < 1 || hidden > kHidMax) return FMP_ERR_INVALID_ARG;
  const size_t H = hidden;
  const size_t n = 2 * in * H + H * H + 2 * H + in;
  if (bytes != n * 4) return FMP_ERR_INVALID_ARG;
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(w[i])) return FMP_ERR_INVALID_ARG;
  const float* W1 = w;
  const float* b1 = W1 + H * in;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + in * H;
  std::vector<uint16_t> w1(H * in), w2(H * H), w3(in * H);
  for (size_t i = 0; i < w1.size(); ++i) w1[i] = to_bf16_bits(W1[i]);
  for (size_t i = 0; i < w2.size(); ++i) w2[i] = to_bf16_bits(W2[i]);
  for (size_t i = 0; i < w3.size(); ++i) w3[i] = to_bf16_bits(W3[i]);
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(h->d_W1, w1.data(), w1.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_W2, w2.data(), w2.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_W3, w3.data(), w3.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_b1, b1, H * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_b2, b2, H * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_b3, b3, in * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    h->err = std::string("fmp_set_coarse_model: ") + hipGetErrorString(e);
    return FMP_ERR_HIP;
  }
  h->hidden = hidden;
  h->learned_set = true;
  return FMP_OK;
}

fmp_status fmp_coarse_restrict(fmp_handle h, const double* r, double* rc, void* stream) {
  if (!h || !r || !rc) return FMP_ERR_INVALID_ARG;
  if (!h->precond_ok) return FMP_ERR_UNSUPPORTED;
  const hipError_t e = restrict_launch(h, r, rc, (hipStream_t)stream);
  if (e != hipSuccess) {
    h->err = std::string("fmp_coarse_restrict: ") + hipGetErrorString(e);
    return FMP_ERR_HIP;
  }
  return FMP_OK;
}

size_t fmp_mlp_scratch_bytes(int32_t in, int32_t H, int32_t B) {
  if (in < 1 || H < 1 || B < 1) return 0;
  const size_t bh = (size_t)B * H * 4, bi = (size_t)B * in * 4;
  return 4 * al(bh) + 2 * al(bi) + al(1024 * 8);
}

fmp_status fmp_mlp_loss_grad(int32_t in, int32_t H, int32_t B, const float* params, const float* X,
                             const float* Y, float* grads, float* loss, void* work,
                             size_t work_bytes, void* stream) {
  if (in < 1 || H < 1 || B < 1 || !params || !X || !Y || !grads || !loss || !work)
    return FMP_ERR_INVALID_ARG;
  if (work_bytes < fmp_mlp_scratch_bytes(in, H, B)) return FMP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const float* W1 = params;
  const float* b1 = W1 + (size_t)H * in;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (size_t)H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + (size_t)in * H;
  float* gW1 = grads;
  float* gb1 = gW1 + (size_t)H * in;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (size_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + (size_t)in * H;
  char* p = (char*)work;
  auto take = [&](size_t bytes) { char* r = p; p += al(bytes); return (float*)r; };
  float* H1 = take((size_t)B * H * 4);
  float* H2 = take((size_t)B * H * 4);
  float* dZ2 = take((size_t)B * H * 4);
  float* dZ1 = take((size_t)B * H * 4);
  float* O = take((size_t)B * in * 4);
  float* dO = take((size_t)B * in * 4);
  double* part = (double*)take(1024 * 8);
  hipError_t e = hipSuccess;
  auto run = [&](GemmArgs g) { if (e == hipSuccess) e = gemm(g, s); };
  // forward
  run({X, in, 1, W1, 1, in, H1, H, 1, B, H, in, b1, 1, nullptr, 0, 0});
  run({H1, H, 1, W2, 1, H, H2, H, 1, B, H, H, b2, 1, nullptr, 0, 0});
  run({H2, H, 1, W3, 1, H, O, in, 1, B, in, H, b3, 0, nullptr, 0, 0});
  const long long no = (long long)B * in;
  const int nb = 1024;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kT), 0, s, O, Y, no, (float)(1.0 / (double)no), dO, part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, s, part, nb, 1.0 / (double)no, loss);
    e = hipGetLastError();
  }
  // backward
  run({dO, 1, in, H2, H, 1, gW3, H, 1, in, H, B, nullptr, 0, nullptr, 0, 0});      // dW3 = dO^T H2
  run({dO, in, 1, W3, H, 1, dZ2, H, 1, B, H, in, nullptr, 0, H2, H, 1});           // dZ2
  run({dZ2, 1, H, H1, H, 1, gW2, H, 1, H, H, B, nullptr, 0, nullptr, 0, 0});       // dW2 = dZ2^T H1
  run({dZ2, H, 1, W2, H, 1, dZ1, H, 1, B, H, H, nullptr, 0, H1, H, 1});            // dZ1
  run({dZ1, 1, H, X, in, 1, gW1, in, 1, H, in, B, nullptr, 0, nullptr, 0, 0});     // dW1 = dZ1^T X
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_colsum, dim3((in + kT - 1) / kT), dim3(kT), 0, s, dO, B, in, gb3);
    hipLaunchKernelGGL(k_colsum, dim3((H + kT - 1) / kT), dim3(kT), 0, s, dZ2, B, H, gb2);
    hipLaunchKernelGGL(k_colsum, dim3((H + kT - 1) / kT), dim3(kT), 0, s, dZ1, B, H, gb1);
    e = hipGetLastError();
  }
  return e == hipSuccess ? FMP_OK : FMP_ERR_HIP;
}

// Device address of `scratch` on the current GPU, looked up on the first call
// made with that GPU current and kept per device ordinal.
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

static fmp_status static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fmp_set_free_error("fmp_mlp_loss_grad_noalloc: no current HIP device");
    return FMP_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fmp_set_free_error(std::string("fmp_mlp_loss_grad_noalloc: hipGetSymbolAddress: ") +
                         hipGetErrorString(e));
      return FMP_ERR_HIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FMP_OK;
}

fmp_status fmp_mlp_loss_grad_noalloc(int32_t in, int32_t H, int32_t B, const float* params,
                                     const float* X, const float* Y, float* grads, float* loss,
                                     void* stream) {
  if (in < 1 || H < 1 || B < 1 || !params || !X || !Y || !grads || !loss)
    return FMP_ERR_INVALID_ARG;
  const size_t need = fmp_mlp_scratch_bytes(in, H, B);
  if (need > kMlpStaticScratchBytes) {
    fmp_set_free_error("fmp_mlp_loss_grad_noalloc: the shapes need " + std::to_string(need) +
                       " bytes of scratch, more than the " +
                       std::to_string(kMlpStaticScratchBytes) + " bytes of the static buffer");
    return FMP_ERR_WORKSPACE;
  }
  void* p = nullptr;
  const fmp_status st = static_scratch(&p);
  if (st != FMP_OK) return st;
  // every scratch region is written before it is read (layer outputs,
  // gradients, per-block partials), so nothing needs clearing between calls
  return fmp_mlp_loss_grad(in, H, B, params, X, Y, grads, loss, p, kMlpStaticScratchBytes, stream);
}

fmp_status fmp_mlp_adam(int32_t n, float* params, const float* grads, float* m, float* v, int32_t t,
                        float lr, void* stream) {
  if (n < 1 || !params || !grads || !m || !v || t < 1) return FMP_ERR_INVALID_ARG;
  const float bc1 = 1.f - powf(0.9f, (float)t), bc2 = 1.f - powf(0.999f, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((n + kT - 1) / kT), dim3(kT), 0, (hipStream_t)stream, n, params,
                     grads, m, v, lr, bc1, bc2);
  return hipGetLastError() == hipSuccess ? FMP_OK : FMP_ERR_HIP;
}

}  // extern "C"
