// BF16 transform passes on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Same three-pass structure and the same mathematics as the vector-ALU passes
// (Sec. III-A Steps 1-3; Algorithm 1, exact_solve: forward DCT-II/DST-I per
// component, closed-form 3x3 solve of eq. (12) per wavenumber, inverse), with
// every directional contraction a small GEMM on the matrix cores, the form the
// paper gives its transforms (Sec. III-C, GEMM-based discrete transform).
// Operands are bf16 (inputs rounded once when they are staged, tables at
// setup), products accumulate in FP32, the 3x3 solve is FP32.
//
// Fragment layout (16x16x32): lane l holds A[m = l%16][k = 8(l/16) .. +7],
// B[k = 8(l/16) .. +7][n = l%16] and D[m = 4(l/16) + i][n = l%16], i < 4.
// A and B fragments are single 16-byte loads: every operand is stored with
// its K index contiguous (tables row-major [out][in] with row stride 64; LDS
// rows of KP + 8 bf16).  A D fragment holds four consecutive rows of one
// column, which the passes arrange to be four consecutive elements in
// memory, so each lane writes them with one 8-byte store.
//
// Staging W per box component: bf16 chunks of 4 consecutive z values,
// ordered [z / 4][x'][y'] (y' fastest), so that a group of 16 lanes that
// holds 4 z values of 16 consecutive columns reads or writes 128 contiguous
// bytes in every pass.  A box component takes ceil(nz / 4) chunk planes.
// Pass B needs no exchange between waves: a wave owns 16 columns of all three
// components, so the 3x3 solve is done in registers.
//   A  gather 4 z-planes -> x GEMM -> y GEMM -> W (one chunk per lane and tile)
//   B  z GEMM -> solve -> inverse z GEMM, W -> W
//   C  W (one chunk per column) -> inverse y GEMM -> inverse x GEMM -> scatter
// The LDS buffers of passes A and C are zero-filled before they are staged,
// so fragments read rows and K indices beyond the valid ranges as zeros
// without masking; pass B masks its column fragments beyond nz.
#include "fmp_common.h"

namespace fmp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kTB = 96;   // bf16 table row stride (largest class)
constexpr int ZS = 4;     // z planes per pass A / C work item

template <int NP>
struct Geo {
  static constexpr int NT = (NP + 15) / 16;   // 16-wide tiles covering a side
  static constexpr int NR = NT * 16;          // padded side
  static constexpr int KS = (NP + 31) / 32;   // k-steps of 32
  static constexpr int KP = KS * 32;          // padded K
  static constexpr int RS = KP + 8;           // LDS row stride (bf16): spreads banks
};

__device__ __forceinline__ f32x4 mma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

__device__ __forceinline__ bf16x8 zero8() {
  const __bf16 z = (__bf16)0.f;
  return bf16x8{z, z, z, z, z, z, z, z};
}

__device__ __forceinline__ bf16x4 zero4() {
  const __bf16 z = (__bf16)0.f;
  return bf16x4{z, z, z, z};
}

__device__ __forceinline__ bf16x4 pack4(const f32x4& v) {
  return bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
}

__device__ __forceinline__ bool box_wall(int q, int x, int y, int z) {
  return q == 0 ? (y == 0 || z == 0) : (q == 1 ? (x == 0 || z == 0) : (x == 0 || y == 0));
}

// one 16 x 16 output tile: sum over the k-steps of A(ks) x B(ks)
template <int KS, class FA, class FB>
__device__ __forceinline__ f32x4 tile_mma(FA a, FB b) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) acc = mma(a(ks), b(ks), acc);
  return acc;
}

// table fragments for all output tiles: f[nt][ks] = T[16 nt + l%16][32 ks + 8(l/16) ..]
template <int NT, int KS>
__device__ __forceinline__ void load_tab(bf16x8 (&f)[NT][KS], const __bf16* T, int l16, int g) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) f[nt][ks] = ld8(T + (nt * 16 + l16) * kTB + 32 * ks + 8 * g);
}

template <int KS>
__device__ __forceinline__ f32x4 tile_frag(const bf16x8 (&a)[KS], const bf16x8 (&b)[KS]) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) acc = mma(a[ks], b[ks], acc);
  return acc;
}

// zero the elements of a fragment whose K index k0 + e is not below n
__device__ __forceinline__ bf16x8 kmask(bf16x8 v, int k0, int n) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 u = __builtin_bit_cast(u32x4, v);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int k = k0 + 2 * d;
    u[d] &= (k + 1 < n) ? 0xFFFFFFFFu : ((k < n) ? 0x0000FFFFu : 0u);
  }
  return __builtin_bit_cast(bf16x8, u);
}

// A fragments of this wave's NT row tiles (wave + 4 j) of an LDS operand
// whose padding (rows and K indices beyond the valid ranges) holds zeros
template <int NT, int KS, int RS>
__device__ __forceinline__ void load_rows_padded(bf16x8 (&a)[NT][KS], const __bf16* L, int wave,
                                                 int l16, int g) {
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int row = (wave + 4 * j) * 16 + l16;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) a[j][ks] = ld8(L + row * RS + 32 * ks + 8 * g);
  }
}

// zero n bf16 (a multiple of 8) of LDS with 16-byte stores
template <int N>
__device__ __forceinline__ void zero_lds(__bf16* L, int t) {
  static_assert(N % 8 == 0, "whole 16-byte chunks");
#pragma unroll
  for (int i = t; i < N / 8; i += 256) *reinterpret_cast<bf16x8*>(L + 8 * i) = zero8();
}

// ---------------------------------------------------------------- pass A
// One LDS buffer of ZS * NR rows, used twice: first the gathered slab
// S[(zl, y)][x] (K = x contiguous), then, after every wave has moved its A
// fragments into registers, the x-transformed slab Y[(p, zl)][y].  Wave w
// owns the row tiles w, w + 4, ... (NT of them) in both GEMMs; table
// fragments are loaded into registers once per block.
template <int NP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NP <= 34 ? 4 : 1))) void k_mpass_a(const double* __restrict__ r, __bf16* __restrict__ W,
                                                 const BoxDev* __restrict__ boxes,
                                                 const DomainDev* __restrict__ doms,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb) {
  using G = Geo<NP>;
  constexpr int NR = G::NR, KS = G::KS, RS = G::RS, NT = G::NT;
  constexpr int ROWS = ZS * NR;
  __shared__ __align__(16) __bf16 S[ROWS * RS];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const DomainDev& D = doms[B.dom];
  const double* src = r + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  bf16x8 tx[NT][KS], ty[NT][KS], a[NT][KS];
  // the slab's padding (rows beyond (nzs, ny), K beyond nx) and later the
  // padding of Y (K beyond NR) must read as zero: fill the buffer first
  zero_lds<ROWS * RS>(S, t);
  __syncthreads();

  {  // S^gamma: the slab's nzs * ny * nx elements, walls as zero; loads first.
     // A thread's elements t + 256 i are stepped from its first one by the
     // fixed increment of 256 elements (two carries), not decomposed anew;
     // the LDS indices are stepped again when the values are committed, so
     // that only the loaded values occupy registers while the loads fly.
    const int plane = ny * nx, tot = nzs * plane;
    const double* s0 = src + ((long long)(B.bz0 + z0) * D.ny + B.by0) * D.nx + B.bx0;
    int zl = t / plane, y = (t - zl * plane) / nx, x = t - zl * plane - y * nx;
    const int dz = 256 / plane, r256 = 256 - dz * plane, dy = r256 / nx, dx = r256 - dy * nx;
    int off = (zl * D.ny + y) * D.nx + x;          // element offset from s0
    int li = (zl * NR + y) * RS + x;               // LDS index
    const int doff = (dz * D.ny + dy) * D.nx + dx, dli = (dz * NR + dy) * RS + dx;
    const int cx_off = D.nx - nx, cx_li = RS - nx;               // x carry
    const int cy_off = (D.ny - ny) * D.nx, cy_li = (NR - ny) * RS; // y carry
    const bool wx = q != 0, wy = q != 1, wz = q != 2;  // slot 0 of a node axis is a wall
    // elements in flight per thread: all of them up to 40, else chunks of 16
    constexpr int NI = (ZS * NP * NP + 255) / 256;
    constexpr int CH = NI <= 40 ? NI : 16;
    constexpr int NCH = (NI + CH - 1) / CH;
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
      double v[CH];
      const int x1 = x, y1 = y, z1 = zl, l1 = li;
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        // 32-bit byte offset from the slab's (uniform) base: one VGPR per
        // address instead of two (setup refuses domains whose 4-plane span
        // reaches 4 GiB)
        const unsigned bo = (unsigned)(t + 256 * (ch * CH + i) < tot ? off : 0) * 8u;
        v[i] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(s0) + bo);
        x += dx; y += dy; off += doff;
        if (x >= nx) { x -= nx; ++y; off += cx_off; }
        if (y >= ny) { y -= ny; off += cy_off; }
      }
      x = x1; y = y1; zl = z1; li = l1;
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        // FP64 -> FP32 -> bf16, each step rounding to nearest even (the empty
        // asm keeps the compiler from fusing the two into one exact rounding,
        // which costs a dozen instructions per element)
        float f = (float)v[i];
        asm("" : "+v"(f));
        const bool wall = (wx && x == 0) || (wy && y == 0) || (wz && z0 + zl == 0);
        if (t + 256 * (ch * CH + i) < tot) S[li] = (__bf16)(wall ? 0.f : f);
        x += dx; y += dy; zl += dz; li += dli;
        if (x >= nx) { x -= nx; ++y; li += cx_li; }
        if (y >= ny) { y -= ny; ++zl; li += cy_li; }
      }
    }
  }
  load_tab(tx, tb + (q == 0 ? B.mdct[0] : B.mdst[0]), l16, g);
  __syncthreads();

  // x: D[(zl, y)][p] = sum_x S[(zl, y)][x] T[p][x]
  load_rows_padded<NT, KS, RS>(a, S, wave, l16, g);
  __syncthreads();                                // S is overwritten by Y from here
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int row = (wave + 4 * j) * 16 + 4 * g, zl = row / NR, y = row - zl * NR;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {             // lane: Y[(p, zl)][y .. y+3]
      const int p = nt * 16 + l16;
      *reinterpret_cast<bf16x4*>(S + (p * ZS + zl) * RS + y) = pack4(tile_frag<KS>(a[j], tx[nt]));
    }
  }
  __syncthreads();

  // y: D[(p, zl)][q'] = sum_y Y[(p, zl)][y] T[q'][y]  ->  chunk z0 / 4 of column (p, q')
  load_tab(ty, tb + (q == 1 ? B.mdct[1] : B.mdst[1]), l16, g);   // one table live at a time
  load_rows_padded<NT, KS, RS>(a, S, wave, l16, g);
  __bf16* Wc = W + B.w_off + (long long)q * box_wvol(B, true) + (long long)(z0 / 4) * ny * nx * 4;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int p = (wave + 4 * j) * 4 + g;         // the lane's rows: (p, zl = 0..3)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int qq = nt * 16 + l16;
      const f32x4 acc = tile_frag<KS>(a[j], ty[nt]);
      if (p < nx && qq < ny) *reinterpret_cast<bf16x4*>(Wc + (p * ny + qq) * 4) = pack4(acc);
    }
  }
}

// ---------------------------------------------------------------- pass B
// Wave w of a block owns the 16 columns c0 + 16 w + (0..15) of all three
// components.  Forward z as D[r][c] = sum_z T[r][z] X[z][c] (table = A,
// column data = B, read straight from W), solve in registers, inverse z as
// D[z][c] = sum_r Ti[z][r] E[r][c] with E restaged through the wave's LDS rows
// (r contiguous per column).
template <int NP>
__global__ __launch_bounds__(256) void k_mpass_b(__bf16* __restrict__ W,
                                                 const BoxDev* __restrict__ boxes,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb,
                                                 const float* __restrict__ sig) {
  using G = Geo<NP>;
  constexpr int NT = G::NT, KS = G::KS, KP = G::KP, RS = G::RS;
  __shared__ __align__(16) __bf16 E[4][3][16][RS];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int nx = B.nx, ny = B.ny, nz = B.nz, nzc = B.wzp / 4;
  const int plane = ny * nx;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int c = wk.y + 16 * wave + l16;
  const bool active = c < plane;
  const long long wv = box_wvol(B, true);
  const __bf16* col0 = W + B.w_off + (long long)min(c, plane - 1) * 4;   // chunk 0 of column c

  // column fragments X[z = 32 ks + 8 g ..][c] (two chunks each), zero beyond nz
  bf16x8 xb[3][KS];
#pragma unroll
  for (int qq = 0; qq < 3; ++qq)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int ch = 8 * ks + 2 * g;
      const bf16x4 lo = ch < nzc ? *reinterpret_cast<const bf16x4*>(col0 + qq * wv + (long long)ch * plane * 4) : zero4();
      const bf16x4 hi = ch + 1 < nzc ? *reinterpret_cast<const bf16x4*>(col0 + qq * wv + (long long)(ch + 1) * plane * 4) : zero4();
      bf16x8 v = bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      xb[qq][ks] = kmask(v, 4 * ch, nz);
    }
  const __bf16* Tst = tb + B.mdst[2];             // DST-I along z (E_x, E_y): symmetric
  const __bf16* Tct = tb + B.mdct[2];             // DCT-II along z (E_z)
  const __bf16* Tci = tb + B.mdctT[2];            // its transpose
  f32x4 acc[3][NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    const int rrow = mt * 16 + l16;
#pragma unroll
    for (int qq = 0; qq < 3; ++qq) {
      const __bf16* T = qq == 2 ? Tct : Tst;
      acc[qq][mt] = tile_mma<KS>([&](int ks) { return ld8(T + rrow * kTB + 32 * ks + 8 * g); },
                                 [&](int ks) { return xb[qq][ks]; });
    }
  }

  // e = (r + alpha s (s.r)) / (1 + alpha |s|^2) at wavenumbers (x, y, r)
  const int cc = active ? c : 0;
  const int xx = cc / ny, yy = cc - xx * ny;          // columns are (x', y'), y' fastest
  const float sx = sig[B.sig[0] + xx], sy = sig[B.sig[1] + yy];
  const float alpha = (float)B.alpha;
  const float sxy2 = __builtin_fmaf(sx, sx, sy * sy);
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = mt * 16 + 4 * g + i;
      const float sz = sig[B.sig[2] + min(rr, nz - 1)];
      const float a = acc[0][mt][i], b = acc[1][mt][i], d = acc[2][mt][i];
      const float dot = __builtin_fmaf(sx, a, __builtin_fmaf(sy, b, sz * d));
      const float inv = 1.f / __builtin_fmaf(alpha, __builtin_fmaf(sz, sz, sxy2), 1.f);
      const float ad = alpha * dot;
      const bool ok = rr < nz;
      acc[0][mt][i] = ok ? __builtin_fmaf(ad, sx, a) * inv : 0.f;
      acc[1][mt][i] = ok ? __builtin_fmaf(ad, sy, b) * inv : 0.f;
      acc[2][mt][i] = ok ? __builtin_fmaf(ad, sz, d) * inv : 0.f;
    }
#pragma unroll
  for (int qq = 0; qq < 3; ++qq) {
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      *reinterpret_cast<bf16x4*>(&E[wave][qq][l16][mt * 16 + 4 * g]) = pack4(acc[qq][mt]);
    if (KP > NT * 16)                             // K padding of the inverse
      *reinterpret_cast<bf16x4*>(&E[wave][qq][l16][NT * 16 + (4 * g) % (KP - NT * 16)]) = zero4();
  }
  __syncthreads();

#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    const int zrow = mt * 16 + l16;
#pragma unroll
    for (int qq = 0; qq < 3; ++qq) {
      const __bf16* T = qq == 2 ? Tci : Tst;
      const f32x4 o = tile_mma<KS>([&](int ks) { return ld8(T + zrow * kTB + 32 * ks + 8 * g); },
                                   [&](int ks) { return ld8(&E[wave][qq][l16][32 * ks + 8 * g]); });
      const int ch = mt * 4 + g;                    // the lane's rows: chunk ch of column c
      if (active && ch < nzc)
        *reinterpret_cast<bf16x4*>(W + B.w_off + qq * wv + ((long long)ch * plane + c) * 4) = pack4(o);
    }
  }
}

// ---------------------------------------------------------------- pass C
// One LDS buffer used twice, as in pass A: the slab X[(p, zl)][q'] (K = q',
// the spectral y index), then U[(y, zl)][p] after the inverse y GEMM (K = p,
// the spectral x index).
template <int NP>
__global__ __launch_bounds__(256) void k_mpass_c(const __bf16* __restrict__ W, double* __restrict__ z,
                                                 const BoxDev* __restrict__ boxes,
                                                 const DomainDev* __restrict__ doms,
                                                 const int4* __restrict__ work,
                                                 const __bf16* __restrict__ tb,
                                                 const double* __restrict__ coarse, int nsub) {
  using G = Geo<NP>;
  constexpr int NR = G::NR, KS = G::KS, RS = G::RS, NT = G::NT;
  constexpr int ROWS = ZS * NR;
  __shared__ __align__(16) __bf16 X[ROWS * RS];
  const int4 wk = work[xcd_remap(blockIdx.x, gridDim.x)];
  const BoxDev& B = boxes[wk.x];
  const int q = wk.y, z0 = wk.z;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int nzs = min(ZS, nz - z0);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int lz0 = B.oz0 - B.bz0, lz1 = lz0 + B.sz;
  const int ly0 = B.oy0 - B.by0, ly1 = ly0 + B.sy;
  const int lx0 = B.ox0 - B.bx0, lx1 = lx0 + B.sx;
  if (z0 + ZS <= lz0 || z0 >= lz1) return;         // no owned plane in this slab
  bf16x8 ty[NT][KS], tx[NT][KS], a[NT][KS];
  // rows p >= nx and K indices beyond ny of X, and K beyond NR of U, must
  // read as zero: fill the buffer first
  zero_lds<ROWS * RS>(X, t);
  __syncthreads();

  {  // chunk z0 / 4 of the slab's columns (p, q'): X[(p, zl)][q'], two
     // neighbouring columns (q', q'+1) per step: one 16-byte read of W and
     // 4-byte LDS stores (column ny, when ny is odd, is masked on reading)
    const int plane = ny * nx, npair = (ny + 1) >> 1;
    const __bf16* Wc = W + B.w_off + (long long)q * box_wvol(B, true) + (long long)(z0 / 4) * plane * 4;
    const float inv_np = 1.f / (float)npair;
    for (int e = t; e < nx * npair; e += 256) {
      const int p = (int)(((float)e + 0.5f) * inv_np), qq = 2 * (e - p * npair);
      const __bf16* src = Wc + (p * ny + qq) * 4;
      const bf16x4 v0 = *reinterpret_cast<const bf16x4*>(src);
      const bf16x4 v1 = qq + 1 < ny ? *reinterpret_cast<const bf16x4*>(src + 4) : zero4();
#pragma unroll
      for (int zl = 0; zl < ZS; ++zl) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        *reinterpret_cast<bf16x2*>(X + (p * ZS + zl) * RS + qq) = bf16x2{v0[zl], v1[zl]};
      }
    }
  }
  load_tab(ty, tb + (q == 1 ? B.mdctT[1] : B.mdst[1]), l16, g);
  __syncthreads();

  // inverse y: D[(p, zl)][m] = sum_q' X[(p, zl)][q'] Ti[m][q']; rows p >= nx read as zero
  load_rows_padded<NT, KS, RS>(a, X, wave, l16, g);
  __syncthreads();                                // X is overwritten by U from here
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int p = (wave + 4 * j) * 4 + g;         // the lane's rows: (p, zl = 0..3)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int m = nt * 16 + l16;
      const f32x4 acc = tile_frag<KS>(a[j], ty[nt]);
#pragma unroll
      for (int zl = 0; zl < ZS; ++zl) X[(m * ZS + zl) * RS + p] = (__bf16)acc[zl];
    }
  }
  __syncthreads();

  // inverse x: D[(y, zl)][l] = sum_p U[(y, zl)][p] Ti[l][p], then S^0T
  load_tab(tx, tb + (q == 0 ? B.mdctT[0] : B.mdst[0]), l16, g);
  load_rows_padded<NT, KS, RS>(a, X, wave, l16, g);
  const DomainDev& D = doms[B.dom];
  double* dst = z + D.offset + (long long)q * D.nz * D.ny * D.nx;
  const double cq = coarse ? coarse[(long long)q * nsub + B.sub] : 0.0;
  const long long pz = (long long)D.ny * D.nx;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int y = (wave + 4 * j) * 4 + g;         // the lane's rows: (y, zl = 0..3)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int x = nt * 16 + l16;
      const f32x4 acc = tile_frag<KS>(a[j], tx[nt]);
      if (y < ly0 || y >= ly1 || x < lx0 || x >= lx1) continue;
      const int gy = B.by0 + y, gx = B.bx0 + x;
      double* col = dst + ((long long)(B.bz0 + z0) * D.ny + gy) * D.nx + gx;   // (z0, y, x)
#pragma unroll
      for (int zl = 0; zl < ZS; ++zl) {
        const int lz = z0 + zl;
        if (zl >= nzs || lz < lz0 || lz >= lz1) continue;
        double val = (double)acc[zl];
        if (coarse && !box_wall(q, gx, gy, B.bz0 + lz)) val += cq;
        col[(long long)zl * pz] = val;
      }
    }
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
    case 8: CALL(64); break;                            \
    case 9: CALL(96); break;                            \
    default: return hipErrorInvalidValue;               \
  }

}  // namespace

int mfma_zslab(int) { return ZS; }

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
