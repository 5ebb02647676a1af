// Internal declarations shared by the FlashMP HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "flashmp.h"

namespace fmp {

// Largest box side with a compiled transform class (the matrix-core passes),
// the largest side of the vector-ALU passes (FP64 / FP32), and the row stride
// of every full transform table (stored kTS x kTS, zero padded).
constexpr int kMaxSide = 96;
constexpr int kMaxSideVec = 48;
constexpr int kTS = 96;
constexpr int kHS = 24;   // stride of the half (butterfly) tables, sides <= kMaxSideVec
constexpr int kHL = 48;   // stride of the half tables of the larger sides (<= kTS)

// Transform size classes: a box of largest side n runs the kernels compiled
// for the smallest class >= n (zero-padded rows/columns cost flops only).
// Classes above kMaxSideVec exist on the matrix-core (BF16) path only.
constexpr int kClasses[] = {8, 16, 24, 26, 32, 34, 40, 48, 64, 96};
constexpr int kNumClasses = sizeof(kClasses) / sizeof(kClasses[0]);

struct DomainDev {
  int nx, ny, nz;
  int eps_b;            // permittivity cube side (0 = eps 1)
  long long offset;     // element offset of this domain's block in a vector
  double c;
  int eps_off;          // offset into the eps table array
  int eps_nbx, eps_nby, eps_nbz;
  int sx, sy, sz;       // owned subdomain sides
  int px, py, pz;       // subdomains per axis
  int sub0;             // global index of the domain's first subdomain
};

// One RAS box.  Table offsets index the per-precision table arrays:
// dct[a] / dst[a] are kTS x kTS matrices for the box side along axis a
// (dctT[a] the transposed DCT-II; DST-I is symmetric), sig[a] the singular
// values sigma_m = 2 sin(m pi / (2 n)).
struct BoxDev {
  int dom;
  int bx0, by0, bz0;    // box origin (cells, in the domain)
  int nx, ny, nz;       // box sides
  int ox0, oy0, oz0;    // owned block origin
  int sx, sy, sz;       // owned block sides
  int sub;              // global subdomain index (coarse vector entry)
  int dct[3], dctT[3], dst[3], sig[3];
  int mdct[3], mdctT[3], mdst[3];   // bf16 tables (row stride 64) of the MFMA passes
  int half[3][2];       // butterfly half tables per axis: [a][0] DCT-II, [a][1] DST-I
  long long w_off;      // staging offset (elements) of component 0
  long long vol;        // nx*ny*nz
  double alpha;         // c / mean eps over the owned block
  int wzp;              // MFMA staging: nz rounded up to 4 (chunks of 4 z values)
  int pad_;
  // index-block subdomains (low-rank boundary correction) only:
  int ibt[3];           // per axis: offset of the side's compact-difference tables
  int wall;             // bit a: the box starts at the PEC wall along axis a
  int corr;             // correction matrix of the box
  int m;                // boundary slots (columns of Q)
  int qoff;             // offset of the box shape's boundary slot list
  int pad2_;
  long long g_off;      // offset of the box's boundary vectors Q^T E, C^{-1} Q^T E
};

// Index-block tables, per distinct side n (row stride kIT, zero padded):
// [0] forward along the half-point axis (U^T), [1] its inverse (U),
// [2] forward along a node axis (V^T), [3] its inverse (V), [4] sigma.
constexpr int kIT = 48;
constexpr int kIBMaxSide = 48;
constexpr long long kIBPerSide = 4LL * kIT * kIT + kIT;

// One correction matrix C^{-1} (mp x mp, row-major, padded with the identity).
struct IBCorrDev {
  long long off;
  int m, mp;
};

// Staging elements of one component of a box: dense [z][y][x] for the
// vector-ALU passes, z-fastest padded columns for the MFMA passes.
__host__ __device__ inline long long box_wvol(const BoxDev& B, bool mfma) {
  return mfma ? (long long)B.nx * B.ny * B.wzp : B.vol;
}

// Stencil tile: 64 x TY columns marching over kStencilZC planes of one domain;
// the tile heights fmp_autotune chooses from, and the default.
struct StencilTile {
  int dom, x0, y0, z0;
};

constexpr int kStencilTX = 64, kStencilZC = 64;
constexpr int kStencilTYs[] = {4, 8, 16};
constexpr int kNumStencilTY = 3;
constexpr int kStencilDefault = 1;   // 64 x 8

// Workgroups of a launch are dealt to the 8 XCDs round-robin (block b runs on
// XCD b % 8).  xcd_remap(b, nb) renumbers them so that each XCD works through
// one contiguous run of work items: neighbouring items (adjacent tiles or
// boxes, which read shared halo lines) then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb / 8, r = nb % 8;
  const int x = b % 8, idx = b / 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + idx;
}

// Fixed reduction geometry: stage 1 uses kRedBlocks blocks of 256 threads.
constexpr int kRedBlocks = 1024;
constexpr int kMaxDots = 34;    // CGS: up to restart+1 basis vectors + ||w||^2

// A reduction segment: the elements [e0, e1) of a vector, walked by blocks
// [b0, b0 + nb) of the kRedBlocks grid.  Either one segment covers the whole
// vector (one Krylov method on the concatenated system) or there is one
// segment per domain (independent solves advanced in lockstep).  A segmented
// launch reads a per-block copy of its block's segment; `grp` indexes
// per-segment coefficient and flag arrays.
struct SegDev {
  long long e0, e1;
  int b0, nb;
  int grp, dom;   // dom = the domain holding e0 (walls are masked per domain)
};

// ---- launchers (defined in the .hip files) ---------------------------------
hipError_t launch_curlcurl(int ty, const double* x, double* y, const DomainDev* doms,
                           const StencilTile* tiles, int ntiles, const double* eps,
                           hipStream_t s);

// Transform passes for one size class over a range of work items.
// prec: 0 fp64, 1 fp32 (vector ALU); tables typed accordingly.
hipError_t launch_pass_a(int prec, int cls, const double* r, void* W, const BoxDev* boxes,
                         const DomainDev* doms, const int4* work, int nwork, const void* tab,
                         hipStream_t s);
hipError_t launch_pass_b(int prec, int cls, void* W, const BoxDev* boxes, const int4* work,
                         int nwork, const void* tab, hipStream_t s);
hipError_t launch_pass_c(int prec, int cls, const void* W, double* z, const BoxDev* boxes,
                         const DomainDev* doms, const int4* work, int nwork, const void* tab,
                         const double* coarse, int nsub, hipStream_t s);
int pass_a_zslab(int cls);   // planes per pass-A/C work item for a class

// FP64 / FP32 boxes of the classes above kMaxSideVec: gather, three forward
// and three inverse contractions as tiled GEMMs (items work_l + l0[a], nl[a]
// per axis a: box, component, row tile, column tile), solve, scatter; the
// staging holds two copies of each box.
int large_tile_rows();
int large_tile_cols();
int large_rows(int n);      // rows (virtual, see fmp_large.hip) the contractions tile along an axis of n
hipError_t launch_large(int prec, const double* r, void* W, double* z, const BoxDev* boxes,
                        const DomainDev* doms, const int4* work_a, int na, const int4* work_l,
                        const int* l0, const int* nl, int zs, const void* tab,
                        const double* coarse, int nsub, hipStream_t s);

// BF16 MFMA transform passes (staging W in bf16).
hipError_t launch_mfma_pass_a(int cls, const double* r, void* W, const BoxDev* boxes,
                              const DomainDev* doms, const int4* work, int nwork,
                              const __hip_bfloat16* tab, hipStream_t s);
hipError_t launch_mfma_pass_b(int cls, void* W, const BoxDev* boxes, const int4* work,
                              int nwork, const __hip_bfloat16* tab, const float* sig,
                              hipStream_t s);
hipError_t launch_mfma_pass_c(int cls, const void* W, double* z, const BoxDev* boxes,
                              const DomainDev* doms, const int4* work, int nwork,
                              const __hip_bfloat16* tab, const double* coarse, int nsub,
                              hipStream_t s);
int mfma_zslab(int cls);

// ---- Krylov vector kernels -------------------------------------------------
// Dots <a_i, b_i> for i < n: partials[blk * n + i]; then reduce to out[i].
struct DotPtrs {
  const double* a[8];
  const double* b[8];
};
hipError_t launch_dots(const DotPtrs& p, int n, long long len, double* partials, hipStream_t s);
// Multi-dot per segment g: h_{g,i} = <V_i, w>_g (i < nv) and h_{g,nv} = <w, w>_g;
// V_i = V + i * ldv; map = per-block segments; segments whose act[grp] is 0
// are skipped (partials 0).  act may be null (all active).
hipError_t launch_mdot(const double* V, long long ldv, int nv, const double* w,
                       const SegDev* map, const int* act, double* partials, hipStream_t s);
// Final fixed-order reduction of `n` partial columns into out[0..n); post-op
// codes run on thread 0 after the sums (see fmp_krylov.hip).
hipError_t launch_reduce(const double* partials, int n, double* out, int post, double* S,
                         hipStream_t s);
// Per-segment fixed-order reduction: out[g * ostride + i] for i < n, g < nseg.
hipError_t launch_reduce_seg(const double* partials, int n, const SegDev* segs, int nseg,
                             double* out, int ostride, hipStream_t s);
// w -= sum_i h_{g,i} sc_{g,i} V_i on segment g (h_g = h + grp * hld, same
// stride for sc; sc may be null = 1), partial ||w||^2.
hipError_t launch_mupdate(const double* V, long long ldv, int nv, const double* h,
                          const double* sc, int hld, double* w, const SegDev* map, const int* act,
                          double* partials, hipStream_t s);
// x += sum_i y_{g,i} Z_i on segment g (y_g = y + grp * yld).
hipError_t launch_xupdate(const double* Z, long long ldz, int nz, const double* y, int yld,
                          double* x, const SegDev* map, hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* out,
                        long long len, hipStream_t s);   // out = a x + b y
hipError_t launch_scale_copy(const double* x, double a, double* out, long long len,
                             hipStream_t s);              // out = a x
// out = fac[grp] x on each segment (in place allowed; in place, segments
// with factor 1 are skipped).
hipError_t launch_scale_seg(const double* x, const double* fac, double* out, const SegDev* map,
                            hipStream_t s);
// r = b - y with every PEC-wall slot set to 0, partial ||r||^2 per block;
// map must hold one segment per domain.
hipError_t launch_sub_norm(const double* b, const double* y, double* r, const SegDev* map,
                           const DomainDev* doms, double* partials, hipStream_t s);
// Set the PEC-wall slots of x to 0.
hipError_t launch_zero_walls(double* x, const DomainDev* doms, int ndom, hipStream_t s);
// BiCGSTAB fused steps (scalars live in device array S; see fmp_krylov.hip).
hipError_t launch_bicg_p(const double* r, double* p, const double* v, const double* S,
                         long long len, hipStream_t s);
hipError_t launch_bicg_s(const double* r, const double* v, double* sv, const double* S,
                         long long len, hipStream_t s);
hipError_t launch_bicg_xr(double* x, const double* phat, const double* shat, const double* sv,
                          const double* t, double* r, const double* rhat, const double* S,
                          long long len, double* partials, hipStream_t s);

// ---- index-block subdomains with the low-rank boundary correction ----------
// Exact solve (I + alpha M)^{-1} per box: three passes like the PEC boxes but
// with dense compact-difference bases.  Pass A reads r (gather, wall slots 0)
// or, with Win set, staged box arrays; pass C writes the full box arrays to
// Wdst, or, with z set, z = E - (its result) on the owned unknowns.
int ib_class_np(int cls);
int ib_class_of(int n);
int ib_zslab(int np);
hipError_t launch_ib_a(int np, const double* r, const double* Win, double* W, const BoxDev* boxes,
                       const DomainDev* doms, const int4* work, int nwork, const double* tab,
                       hipStream_t s);
hipError_t launch_ib_b(int np, double* W, const BoxDev* boxes, const int4* work, int nwork,
                       const double* tab, hipStream_t s);
hipError_t launch_ib_c(int np, const double* Wsrc, double* Wdst, const double* E, double* z,
                       const BoxDev* boxes, const DomainDev* doms, const int4* work, int nwork,
                       const double* tab, hipStream_t s);

// Records the detail message that fmp_last_error(NULL) returns on this host
// thread (calls that take no handle).
void fmp_set_free_error(const std::string& msg);

// ---- learned coarse correction ---------------------------------------------
hipError_t launch_coarse_restrict(const double* r, const BoxDev* boxes, int nbox,
                                  const DomainDev* doms, double* rc, hipStream_t s);

}  // namespace fmp
