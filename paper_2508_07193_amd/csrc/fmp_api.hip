// C ABI, plans and Krylov drivers of the FlashMP library (host side).
//
// Setup (fmp_setup_subdomains) splits every domain into owned blocks, extends
// each by the overlap into a PEC box clipped at the walls (the RAS boxes of
// Sec. II-B), builds the DCT-II / DST-I tables of every distinct box side,
// sorts boxes into transform size classes and cuts each class into batches
// whose spectral staging fits the last-level cache.  All device tables live
// in the caller's workspace.
//
// fmp_solve runs right-preconditioned BiCGSTAB or flexible GMRES(m) (the
// solvers of Sec. IV-A) entirely on the device: vector updates, dots and
// scalar recurrences are kernels; the host only reads a few scalars per
// iteration for the stopping test and the small Hessenberg least-squares
// problem.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <memory>

#include "fmp_common.h"
#include "fmp_ctx.h"

using namespace fmp;

namespace {

constexpr size_t kAlign = 256;
constexpr int kTB = 96;         // row stride of the bf16 tables (largest class)
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

constexpr int kScal = 256;      // doubles in the scalar area
constexpr int kScalJ = 200;     // learned-correction residual test: ||v - w||^2, ||v - w + A d||^2
// per-group scalar block (kSD doubles per group)
constexpr int kSD = 192;
constexpr int kSDH = 0;         // h column and ||w||^2 before the update (<= 34)
constexpr int kSDW = 40;        // ||w||^2 after the update
constexpr int kSDY = 48;        // update coefficients y (<= 33)
constexpr int kSDR = 96;        // ||r||^2 of a residual
constexpr int kSDS = 128;       // squared scales s_i^2 of the stored basis (<= 33)

struct Parts {
  int own0, own1, box0, box1;
};

std::vector<Parts> axis_parts(int n, int sub, int overlap) {
  std::vector<Parts> out;
  if (sub <= 0) sub = n;
  for (int a = 0; a < n; a += sub)
    out.push_back({a, a + sub, std::max(0, a - overlap), std::min(n, a + sub + overlap)});
  return out;
}

int class_of(int n) {
  for (int c = 0; c < kNumClasses; ++c)
    if (kClasses[c] >= n) return c;
  return -1;
}

// Cut the class-ordered boxes into batches of at most `batch` boxes of one
// class; assign each box its staging offset inside its batch.  Pass A / C
// work items (box, component, first plane of a z-slab) are ordered per batch
// either box by box (h->slab_order = 0) or by component, then slab, then box
// (1): then neighbouring boxes (x fastest, then y) gather the same slab at
// the same time, so the cache lines they share (the overlap rows, and the
// partial lines at both ends of every 34-cell row) are fetched once into the
// XCD's L2, at the price of more distinct pages in flight.  Returns the
// largest batch's staging size (elements).
// FP64 / FP32 boxes of the classes above the vector-ALU passes' limit run the
// tiled-GEMM path, whose staging keeps two copies of each box.
bool large_class(const fmp_ctx* h, int c) {
  return c >= 0 && h->prec != FMP_BF16 && kClasses[c] > kMaxSideVec;
}

long long plan_batches(fmp_ctx* h, int batch) {
  h->launches.clear();
  h->work_a.clear();
  h->work_l.clear();
  h->batch = batch;
  long long wmax = 0;
  const auto cls_at = [&](size_t i) {
    const BoxDev& B = h->boxes[h->order[i]];
    return class_of(std::max(B.nx, std::max(B.ny, B.nz)));
  };
  for (size_t i0 = 0; i0 < h->order.size();) {
    const int c = cls_at(i0);
    size_t i1 = i0;
    while (i1 < h->order.size() && cls_at(i1) == c && (int)(i1 - i0) < batch) ++i1;
    long long woff = 0;
    int nzmax = 0;
    for (size_t i = i0; i < i1; ++i) {
      BoxDev& B = h->boxes[h->order[i]];
      B.w_off = woff;                 // staging is reused batch after batch
      woff += (large_class(h, c) ? 2 : 1) *
              ((3 * box_wvol(B, h->prec == FMP_BF16) + 7) / 8 * 8);   // 16-byte aligned boxes
      nzmax = std::max(nzmax, B.nz);
    }
    wmax = std::max(wmax, woff);
    const int a0 = (int)h->work_a.size();
    if (c >= 0) {
      const int zs = (h->prec == FMP_BF16) ? mfma_zslab(c) : pass_a_zslab(c);
      if (h->slab_order) {
        for (int q = 0; q < 3; ++q)
          for (int z0 = 0; z0 < nzmax; z0 += zs)
            for (size_t i = i0; i < i1; ++i)
              if (z0 < h->boxes[h->order[i]].nz)
                h->work_a.push_back(make_int4(h->order[i], q, z0, 0));
      } else {
        for (size_t i = i0; i < i1; ++i)
          for (int q = 0; q < 3; ++q)
            for (int z0 = 0; z0 < h->boxes[h->order[i]].nz; z0 += zs)
              h->work_a.push_back(make_int4(h->order[i], q, z0, 0));
      }
      Launch L{c, a0, (int)h->work_a.size() - a0, h->wb0[i0], h->wb0[i1] - h->wb0[i0],
               {0, 0, 0}, {0, 0, 0}};
      if (large_class(h, c)) {
        const int TI = large_tile_rows(), TC = large_tile_cols();
        for (int a = 0; a < 3; ++a) {
          L.l0[a] = (int)h->work_l.size();
          for (size_t i = i0; i < i1; ++i) {
            const BoxDev& B = h->boxes[h->order[i]];
            const int n = a == 0 ? B.nx : (a == 1 ? B.ny : B.nz);
            const long long ncol = B.vol / n;
            for (int q = 0; q < 3; ++q)
              for (int it = 0; it * TI < large_rows(n); ++it)
                for (long long ct = 0; ct * TC < ncol; ++ct)
                  h->work_l.push_back(make_int4(h->order[i], q, it, (int)ct));
          }
          L.nl[a] = (int)h->work_l.size() - L.l0[a];
        }
      }
      h->launches.push_back(L);
    }
    i0 = i1;
  }
  return wmax;
}

// Orthonormal DCT-II (rows p, columns l) and DST-I embedded in an n x n
// block (row/column 0 zero), both stored with row stride kTS; sigma_m.
void basis_tables(int n, std::vector<double>& dct, std::vector<double>& dst,
                  std::vector<double>& sig) {
  dct.assign(kTS * kTS, 0.0);
  dst.assign(kTS * kTS, 0.0);
  sig.assign(kTS, 0.0);
  const double sc = sqrt(2.0 / n);
  for (int p = 0; p < n; ++p)
    for (int l = 0; l < n; ++l) {
      // cos(pi p (2l+1) / (2n)) with the integer angle reduced mod 4n
      const long a = (long)p * (2 * l + 1) % (4L * n);
      double v = sc * cos(M_PI * (double)a / (2.0 * n));
      if (p == 0) v = 1.0 / sqrt((double)n);
      dct[p * kTS + l] = v;
    }
  for (int m = 1; m < n; ++m)
    for (int l = 1; l < n; ++l) {
      const long a = (long)m * l % (2L * n);
      dst[m * kTS + l] = sc * sin(M_PI * (double)a / (double)n);
    }
  for (int m = 0; m < n; ++m) sig[m] = 2.0 * sin(M_PI * m / (2.0 * n));
}

bool overlaps(const void* a, const void* b, long long bytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bytes && pb < pa + bytes;
}

fmp_status hip_fail(fmp_ctx* h, hipError_t e, const char* what) {
  if (h) h->err = std::string(what) + ": " + hipGetErrorString(e);
  return FMP_ERR_HIP;
}

#define HIPCHK(h, call)                                  \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return hip_fail(h, _e, #call); \
  } while (0)

uint16_t to_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;   // round to nearest even
  return (uint16_t)(u >> 16);
}

}  // namespace

// ============================================================== precond / spmv
static fmp_status precond_launches(fmp_ctx* h, const double* r, double* z, hipStream_t s,
                                   const double* coarse);

// Replay (or capture, on first use of this (r, z) pair) the launch sequence of
// one apply as a hipGraph.  Capture runs on the handle's private stream; the
// instantiated graph is launched on the caller's stream.
static fmp_status precond_apply(fmp_ctx* h, const double* r, double* z, hipStream_t s,
                                const double* coarse) {
  if (!h->use_graph) return precond_launches(h, r, z, s, coarse);
  for (const auto& g : h->graphs)
    if (g.r == r && g.z == z && g.coarse == (coarse != nullptr)) {
      HIPCHK(h, hipGraphLaunch(g.exec, s));
      return FMP_OK;
    }
  if (h->graphs.size() >= 64) return precond_launches(h, r, z, s, coarse);
  if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const fmp_status st = precond_launches(h, r, z, h->cap_stream, coarse);
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
  if (st != FMP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(h, ei, "hipGraphInstantiate");
  h->graphs.push_back({r, z, coarse != nullptr, exec});
  HIPCHK(h, hipGraphLaunch(exec, s));
  return FMP_OK;
}

static fmp_status precond_launches(fmp_ctx* h, const double* r, double* z, hipStream_t s,
                                   const double* coarse) {
  if (h->ib.on) return ib_apply(h, r, z, s);
  const int prec = h->prec;
  // Several batches: batch k runs on private stream k % ns with staging
  // buffer k % ns, so the passes of up to ns batches overlap.  Batches write
  // disjoint parts of z.
  const int ns = std::min(std::min(h->nstreams, h->n_wbuf), (int)h->launches.size());
  hipStream_t bs[fmp_ctx::kMaxStreams];
  for (int i = 0; i < fmp_ctx::kMaxStreams; ++i) bs[i] = s;
  if (ns > 1) {
    if (!h->ev_fork) HIPCHK(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    for (int i = 0; i < ns; ++i) {
      if (!h->bat_stream[i])
        HIPCHK(h, hipStreamCreateWithFlags(&h->bat_stream[i], hipStreamNonBlocking));
      if (!h->ev_join[i])
        HIPCHK(h, hipEventCreateWithFlags(&h->ev_join[i], hipEventDisableTiming));
    }
    HIPCHK(h, hipEventRecord(h->ev_fork, s));
    for (int i = 0; i < ns; ++i) {
      HIPCHK(h, hipStreamWaitEvent(h->bat_stream[i], h->ev_fork, 0));
      bs[i] = h->bat_stream[i];
    }
  }
  for (size_t k = 0; k < h->launches.size(); ++k) {
    const Launch& L = h->launches[k];
    const int slot = ns > 1 ? (int)(k % ns) : 0;
    const hipStream_t st = bs[slot];
    void* W = h->d_Wk[slot];
    if (large_class(h, L.cls)) {
      HIPCHK(h, launch_large(prec, r, W, z, h->d_boxes, h->d_doms, h->d_work_a + L.a0, L.na,
                             h->d_work_l, L.l0, L.nl, pass_a_zslab(L.cls), h->d_tab, coarse,
                             h->nsub, st));
    } else if (prec == FMP_BF16) {
      HIPCHK(h, launch_mfma_pass_a(L.cls, r, W, h->d_boxes, h->d_doms,
                                   h->d_work_a + L.a0, L.na, (const __hip_bfloat16*)h->d_tab, st));
      HIPCHK(h, launch_mfma_pass_b(L.cls, W, h->d_boxes, h->d_work_b + L.b0, L.nb,
                                   (const __hip_bfloat16*)h->d_tab, h->d_sig32, st));
      HIPCHK(h, launch_mfma_pass_c(L.cls, W, z, h->d_boxes, h->d_doms,
                                   h->d_work_a + L.a0, L.na, (const __hip_bfloat16*)h->d_tab,
                                   coarse, h->nsub, st));
    } else {
      HIPCHK(h, launch_pass_a(prec, L.cls, r, W, h->d_boxes, h->d_doms, h->d_work_a + L.a0,
                              L.na, h->d_tab, st));
      HIPCHK(h, launch_pass_b(prec, L.cls, W, h->d_boxes, h->d_work_b + L.b0, L.nb,
                              h->d_tab, st));
      HIPCHK(h, launch_pass_c(prec, L.cls, W, z, h->d_boxes, h->d_doms, h->d_work_a + L.a0,
                              L.na, h->d_tab, coarse, h->nsub, st));
    }
  }
  if (ns > 1) {
    for (int i = 0; i < ns; ++i) {
      HIPCHK(h, hipEventRecord(h->ev_join[i], bs[i]));
      HIPCHK(h, hipStreamWaitEvent(s, h->ev_join[i], 0));
    }
  }
  return FMP_OK;
}

static fmp_status spmv(fmp_ctx* h, const double* x, double* y, hipStream_t s) {
  HIPCHK(h, launch_curlcurl(kStencilTYs[h->stencil_v], x, y, h->d_doms, h->d_tiles, h->ntiles,
                            h->d_eps, s));
  return FMP_OK;
}

// Learned part: defined in fmp_coarse.hip (returns the device correction
// vector to add in pass C, or nullptr when the model is not set).
fmp_status fmp_coarse_forward(fmp_ctx* h, const double* r, hipStream_t s, const double** out);
hipError_t fmp_coarse_resid_test(fmp_ctx* h, const double* v, const double* w, double* partials,
                            hipStream_t s);
size_t fmp_coarse_workspace(int nsub, int hidden_max);
void fmp_coarse_bind(fmp_ctx* h, void* base);

// ---- persistent autotuner cache ---------------------------------------------
// Key: what the plan's timing depends on (library revision, device, precision,
// overlap, learned part, and every domain's size and subdomain split).
static std::string tune_key(const fmp_ctx* h) {
  std::string k = "flashmp-plan-2";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    k += std::string("|") + prop.gcnArchName;
  k += "|p" + std::to_string(h->prec) + "|o" + std::to_string(h->overlap) + "|l" +
       std::to_string((int)h->use_learned);
  for (const DomainDev& D : h->doms)
    k += "|" + std::to_string(D.nx) + "x" + std::to_string(D.ny) + "x" + std::to_string(D.nz) +
         "/" + std::to_string(D.sx) + "x" + std::to_string(D.sy) + "x" + std::to_string(D.sz);
  for (char& c : k)
    if (c == ' ' || c == '\n' || c == '\t') c = '_';
  return k;
}

static bool tune_cache_find(const char* path, const std::string& key, int* batch, int* ns,
                            int* slab, int* ty) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char line[8192];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[8192];
    int b, n, so, t;
    if (sscanf(line, "%8191s %d %d %d %d", k, &b, &n, &so, &t) == 5 && key == k &&
        b > 0 && n >= 1 && n <= fmp_ctx::kMaxStreams && (so == 0 || so == 1)) {
      bool ty_ok = false;
      for (int v = 0; v < kNumStencilTY; ++v) ty_ok = ty_ok || kStencilTYs[v] == t;
      if (ty_ok) {                                // the last matching record wins
        *batch = b; *ns = n; *slab = so; *ty = t;
        found = true;
      }
    }
  }
  fclose(f);
  return found;
}

static void tune_cache_add(const char* path, const std::string& key, int batch, int ns, int slab,
                           int ty) {
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %d\n", key.c_str(), batch, ns, slab, ty);
  fclose(f);
}

// Detail of the last failed call that has no handle, per host thread.
static thread_local std::string g_free_err;
void fmp::fmp_set_free_error(const std::string& msg) { g_free_err = msg; }

extern "C" {

const char* fmp_status_string(fmp_status st) {
  switch (st) {
    case FMP_OK: return "ok";
    case FMP_NOT_CONVERGED: return "not converged";
    case FMP_ERR_INVALID_ARG: return "invalid argument";
    case FMP_ERR_ALIAS: return "input and output overlap";
    case FMP_ERR_WORKSPACE: return "workspace missing or too small";
    case FMP_ERR_HIP: return "HIP runtime error";
    case FMP_ERR_BREAKDOWN: return "Krylov breakdown or non-finite value";
    case FMP_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* fmp_last_error(fmp_handle h) { return h ? h->err.c_str() : g_free_err.c_str(); }

fmp_status fmp_runtime_version(int32_t* compiled, int32_t* running) {
  if (!compiled || !running) return FMP_ERR_INVALID_ARG;
  *compiled = HIP_VERSION;
  int rt = 0;
  const hipError_t e = hipRuntimeGetVersion(&rt);
  *running = e == hipSuccess ? rt : 0;
  return e == hipSuccess ? FMP_OK : FMP_ERR_HIP;
}

fmp_status fmp_setup_subdomains(const fmp_domain_desc* domains, int32_t n_domains,
                                const fmp_precond_desc* pd, void* ws, size_t* ws_bytes,
                                void* stream, fmp_handle* out) {
  if (!domains || n_domains < 1 || !pd || !ws_bytes) return FMP_ERR_INVALID_ARG;
  if (pd->subdomain != 0 && pd->subdomain != 1) return FMP_ERR_INVALID_ARG;
  const bool index_blocks = pd->subdomain == 1;
  // PEC boxes need an overlap of at least one cell: with none, the owned
  // interface unknowns would sit on box walls and never be corrected
  if (pd->overlap < (index_blocks ? 0 : 1)) return FMP_ERR_INVALID_ARG;
  if (pd->precision < FMP_FP64 || pd->precision > FMP_BF16) return FMP_ERR_INVALID_ARG;
  // the index-block path is FP64, without the learned part or the autotuner
  if (index_blocks && (pd->precision != FMP_FP64 || pd->use_learned || pd->batch_boxes < 0))
    return FMP_ERR_UNSUPPORTED;
  if (out) *out = nullptr;
  std::unique_ptr<fmp_ctx> h(new fmp_ctx());
  h->prec = pd->precision;
  h->overlap = pd->overlap;
  h->use_learned = pd->use_learned != 0;
  h->use_graph = pd->use_graph != 0;

  // ---- domains, boxes, eps tables
  std::vector<double> eps_all;
  long long off = 0;
  std::vector<int> sides_used(kMaxSide + 1, 0);
  for (int d = 0; d < n_domains; ++d) {
    const fmp_domain_desc& D = domains[d];
    if (D.nx < 2 || D.ny < 2 || D.nz < 2 || !(D.c >= 0.0) || !isfinite(D.c))
      return FMP_ERR_INVALID_ARG;
    if (h->prec == FMP_BF16 && 4LL * D.ny * D.nx >= (1LL << 29)) {
      // the bf16 gather addresses a 4-plane slab by 32-bit byte offsets
      h->err = "bf16 transforms need planes of fewer than 2^27 cells";
      return FMP_ERR_UNSUPPORTED;
    }
    const int sub[3] = {D.sub_x > 0 ? D.sub_x : D.nx, D.sub_y > 0 ? D.sub_y : D.ny,
                        D.sub_z > 0 ? D.sub_z : D.nz};
    const int nn[3] = {D.nx, D.ny, D.nz};
    for (int a = 0; a < 3; ++a)
      if (sub[a] < 1 || nn[a] % sub[a]) return FMP_ERR_INVALID_ARG;
    DomainDev dd{};
    dd.nx = D.nx; dd.ny = D.ny; dd.nz = D.nz;
    dd.offset = off;
    dd.c = D.c;
    dd.eps_b = 0;
    int nbx = 0, nby = 0, nbz = 0;
    if (D.eps_block) {
      const int b = D.eps_block_size;
      if (b < 1) return FMP_ERR_INVALID_ARG;
      nbx = (D.nx + b - 1) / b; nby = (D.ny + b - 1) / b; nbz = (D.nz + b - 1) / b;
      dd.eps_b = b;
      dd.eps_off = (int)eps_all.size();
      dd.eps_nbx = nbx; dd.eps_nby = nby; dd.eps_nbz = nbz;
      for (long long i = 0; i < (long long)nbx * nby * nbz; ++i) {
        const double e = D.eps_block[i];
        if (!(e > 0.0) || !isfinite(e)) return FMP_ERR_INVALID_ARG;
        eps_all.push_back(e);
      }
    }
    dd.sx = sub[0]; dd.sy = sub[1]; dd.sz = sub[2];
    dd.px = D.nx / sub[0]; dd.py = D.ny / sub[1]; dd.pz = D.nz / sub[2];
    dd.sub0 = h->nsub;
    h->doms.push_back(dd);
    h->offsets.push_back(off);
    off += 3LL * D.nx * D.ny * D.nz;

    const auto px = axis_parts(D.nx, sub[0], pd->overlap);
    const auto py = axis_parts(D.ny, sub[1], pd->overlap);
    const auto pz = axis_parts(D.nz, sub[2], pd->overlap);
    for (const Parts& Z : pz)
      for (const Parts& Y : py)
        for (const Parts& X : px) {
          BoxDev B{};
          B.dom = d;
          B.bx0 = X.box0; B.by0 = Y.box0; B.bz0 = Z.box0;
          B.nx = X.box1 - X.box0; B.ny = Y.box1 - Y.box0; B.nz = Z.box1 - Z.box0;
          B.ox0 = X.own0; B.oy0 = Y.own0; B.oz0 = Z.own0;
          B.sx = X.own1 - X.own0; B.sy = Y.own1 - Y.own0; B.sz = Z.own1 - Z.own0;
          B.sub = h->nsub++;
          B.vol = (long long)B.nx * B.ny * B.nz;
          B.wzp = (B.nz + 3) / 4 * 4;
          if (std::min(B.nx, std::min(B.ny, B.nz)) < 2) return FMP_ERR_INVALID_ARG;
          const int side_max = std::max(B.nx, std::max(B.ny, B.nz));
          if (side_max > kMaxSide || (index_blocks && side_max > kIBMaxSide))
            h->precond_ok = false;
          else
            sides_used[B.nx] = sides_used[B.ny] = sides_used[B.nz] = 1;
          // alpha = c / mean eps over the owned cells
          double alpha = D.c;
          if (D.eps_block) {
            long double acc = 0.0L;
            const int b = D.eps_block_size;
            for (int k = Z.own0; k < Z.own1; ++k)
              for (int j = Y.own0; j < Y.own1; ++j)
                for (int i = X.own0; i < X.own1; ++i)
                  acc += D.eps_block[((long long)(k / b) * nby + j / b) * nbx + i / b];
            const double mean = (double)(acc / ((long double)B.sx * B.sy * B.sz));
            alpha = D.c / mean;
          }
          B.alpha = alpha;
          h->boxes.push_back(B);
        }
  }
  h->offsets.push_back(off);
  h->len = off;
  if (index_blocks && h->precond_ok) {
    const fmp_status st = ib_prepare(h.get());
    if (st != FMP_OK) return st;
    std::fill(sides_used.begin(), sides_used.end(), 0);   // no PEC-box tables
  }
  if (n_domains > kRedBlocks) {
    h->err = "more domains than reduction blocks (1024)";
    return FMP_ERR_UNSUPPORTED;
  }
  for (int d = 0; d < n_domains; ++d)
    if (h->offsets[d + 1] - h->offsets[d] >= (1LL << 31)) return FMP_ERR_UNSUPPORTED;

  // ---- reduction segments: blocks dealt to domains in proportion to size,
  // at least one each, kRedBlocks in total
  std::vector<SegDev> map_glob(kRedBlocks), segs_dom(n_domains), map_dom(kRedBlocks);
  {
    const SegDev g{0, h->len, 0, kRedBlocks, 0, 0};
    std::fill(map_glob.begin(), map_glob.end(), g);
    std::vector<int> nb(n_domains);
    int tot = 0;
    for (int d = 0; d < n_domains; ++d) {
      const long long ld = h->offsets[d + 1] - h->offsets[d];
      h->seg_len.push_back(ld);
      nb[d] = std::max(1, (int)((double)kRedBlocks * (double)ld / (double)h->len));
      tot += nb[d];
    }
    while (tot > kRedBlocks) {   // take from the domain with the most blocks
      int k = (int)(std::max_element(nb.begin(), nb.end()) - nb.begin());
      --nb[k]; --tot;
    }
    while (tot < kRedBlocks) {   // give to the domain with the most elements per block
      int k = 0;
      for (int d = 1; d < n_domains; ++d)
        if ((double)h->seg_len[d] / nb[d] > (double)h->seg_len[k] / nb[k]) k = d;
      ++nb[k]; ++tot;
    }
    int b0 = 0;
    for (int d = 0; d < n_domains; ++d) {
      segs_dom[d] = SegDev{h->offsets[d], h->offsets[d + 1], b0, nb[d], d, d};
      for (int b = b0; b < b0 + nb[d]; ++b) map_dom[b] = segs_dom[d];
      b0 += nb[d];
    }
  }

  // ---- transform tables for each side in use
  std::vector<int> side_slot(kMaxSide + 1, -1);
  int nsides = 0;
  for (int n = 2; n <= kMaxSide; ++n)
    if (sides_used[n]) side_slot[n] = nsides++;
  // per side: dct, dct^T, dst (kTS x kTS), sig (kTS), then butterfly half
  // tables for DCT-II and DST-I (4 each: TS, TD, TS^T, TD^T; hs x hs with
  // hs = kHS up to kMaxSideVec, kHL above)
  const long long per_side = 3LL * kTS * kTS + kTS + 8LL * kHL * kHL;
  const auto half_stride = [](int n) { return n <= kMaxSideVec ? kHS : kHL; };
  std::vector<double> tab64((size_t)(per_side * nsides), 0.0);
  {
    std::vector<double> c, s, g;
    for (int n = 2; n <= kMaxSide; ++n) {
      if (side_slot[n] < 0) continue;
      basis_tables(n, c, s, g);
      double* base = tab64.data() + side_slot[n] * per_side;
      std::copy(c.begin(), c.end(), base);
      for (int i = 0; i < kTS; ++i)
        for (int j = 0; j < kTS; ++j) base[kTS * kTS + i * kTS + j] = c[j * kTS + i];
      std::copy(s.begin(), s.end(), base + 2 * kTS * kTS);
      std::copy(g.begin(), g.end(), base + 3 * kTS * kTS);
      const int hs = half_stride(n);
      for (int tau = 0; tau < 2; ++tau) {
        const std::vector<double>& T = tau == 0 ? c : s;   // full n x n matrix, stride kTS
        double* hb = base + 3 * kTS * kTS + kTS + tau * 4 * hs * hs;
        const int P = (n - tau) / 2, mid = (n - tau) & 1, cm = (n - 1 + tau) / 2;
        for (int k = 0; k < P + mid; ++k) {
          for (int j = 0; j < P; ++j) hb[k * hs + j] = T[(tau + 2 * k) * kTS + tau + j];
          if (mid) hb[k * hs + P] = T[(tau + 2 * k) * kTS + cm];
        }
        for (int k = 0; k < P; ++k)
          for (int j = 0; j < P; ++j) hb[hs * hs + k * hs + j] = T[(tau + 2 * k + 1) * kTS + tau + j];
        for (int i = 0; i < hs; ++i)
          for (int j = 0; j < hs; ++j) {
            hb[2 * hs * hs + i * hs + j] = hb[j * hs + i];
            hb[3 * hs * hs + i * hs + j] = hb[hs * hs + j * hs + i];
          }
      }
    }
  }
  if (!h->precond_ok) h->boxes.clear();   // stencil and unpreconditioned solves only
  for (BoxDev& B : h->boxes) {
    const int sides[3] = {B.nx, B.ny, B.nz};
    for (int a = 0; a < 3; ++a) {
      const int base = (int)(side_slot[sides[a]] * per_side);
      B.dct[a] = base;
      B.dctT[a] = base + kTS * kTS;
      B.dst[a] = base + 2 * kTS * kTS;
      B.sig[a] = base + 3 * kTS * kTS;
      const int hs = half_stride(sides[a]);
      B.half[a][0] = base + 3 * kTS * kTS + kTS;
      B.half[a][1] = base + 3 * kTS * kTS + kTS + 4 * hs * hs;
      const int mbase = side_slot[sides[a]] * 3 * kTB * kTB;
      B.mdct[a] = mbase;
      B.mdctT[a] = mbase + kTB * kTB;
      B.mdst[a] = mbase + 2 * kTB * kTB;
    }
  }
  // bf16 copies for the MFMA passes: Bt[n][k] with row stride kTB (zero padded)
  std::vector<uint16_t> tab16;
  if (h->prec == FMP_BF16) {
    tab16.assign((size_t)nsides * 3 * kTB * kTB, 0);
    for (int n = 2; n <= kMaxSide; ++n) {
      if (side_slot[n] < 0) continue;
      const double* base = tab64.data() + side_slot[n] * per_side;
      uint16_t* mb = tab16.data() + (size_t)side_slot[n] * 3 * kTB * kTB;
      for (int i = 0; i < kTS; ++i)
        for (int j = 0; j < kTS; ++j) {
          mb[i * kTB + j] = to_bf16(base[i * kTS + j]);                              // DCT-II
          mb[kTB * kTB + i * kTB + j] = to_bf16(base[j * kTS + i]);                  // DCT-II^T
          mb[2 * kTB * kTB + i * kTB + j] = to_bf16(base[2 * kTS * kTS + i * kTS + j]);  // DST-I
        }
    }
  }

  // ---- size classes, work lists and batches
  std::vector<int> cls(h->boxes.size());
  for (size_t i = 0; i < h->boxes.size(); ++i) {
    const BoxDev& B = h->boxes[i];
    cls[i] = class_of(std::max(B.nx, std::max(B.ny, B.nz)));
  }
  h->order.resize(h->boxes.size());
  for (size_t i = 0; i < h->order.size(); ++i) h->order[i] = (int)i;
  std::stable_sort(h->order.begin(), h->order.end(), [&](int a, int b) { return cls[a] < cls[b]; });
  std::vector<int4> work_b;
  for (size_t i = 0; i < h->order.size(); ++i) {
    const int bi = h->order[i];
    const BoxDev& B = h->boxes[bi];
    h->wb0.push_back((int)work_b.size());
    if (cls[bi] < 0) continue;
    for (int c0 = 0; c0 < B.nx * B.ny; c0 += 64) work_b.push_back(make_int4(bi, c0, 0, 0));
  }
  h->wb0.push_back((int)work_b.size());
  // batch = -1: keep room for every candidate of fmp_autotune (whole classes)
  h->tunable = pd->batch_boxes < 0;
  int batch = pd->batch_boxes;
  if (batch <= 0) batch = (h->prec == FMP_FP64) ? 128 : 256;
  h->w_cap = plan_batches(h.get(), h->tunable ? (int)h->boxes.size() : batch);
  if (h->tunable) plan_batches(h.get(), batch);
  const long long w_batch_max = h->w_cap;

  // ---- stencil tiles
  // (one list per tile height, back to back)
  std::vector<StencilTile> tiles;
  int tile0[kNumStencilTY];
  for (int v = 0; v < kNumStencilTY; ++v) {
    tile0[v] = (int)tiles.size();
    for (int d = 0; d < n_domains; ++d) {
      const DomainDev& D = h->doms[d];
      for (int z0 = 0; z0 < D.nz; z0 += kStencilZC)
        for (int y0 = 0; y0 < D.ny; y0 += kStencilTYs[v])
          for (int x0 = 0; x0 < D.nx; x0 += kStencilTX) tiles.push_back({d, x0, y0, z0});
    }
    h->ntiles_v[v] = (int)tiles.size() - tile0[v];
  }
  h->ntiles = h->ntiles_v[h->stencil_v];

  // ---- workspace layout
  const size_t tsz = (h->prec == FMP_FP64) ? 8 : (h->prec == FMP_FP32 ? 4 : 2);
  const size_t wsz = (h->prec == FMP_FP64) ? 8 : (h->prec == FMP_FP32 ? 4 : 2);
  size_t cur = 0;
  const size_t o_doms = cur; cur = align_up(cur + h->doms.size() * sizeof(DomainDev));
  const size_t o_boxes = cur; cur = align_up(cur + h->boxes.size() * sizeof(BoxDev));
  const size_t o_tiles = cur; cur = align_up(cur + tiles.size() * sizeof(StencilTile));
  const size_t o_eps = cur; cur = align_up(cur + std::max<size_t>(1, eps_all.size()) * 8);
  const size_t tab_bytes = (h->prec == FMP_BF16) ? tab16.size() * 2 : tab64.size() * tsz;
  const size_t o_tab = cur; cur = align_up(cur + std::max<size_t>(tab_bytes, 1));
  const size_t o_sig32 = cur; cur = align_up(cur + std::max<size_t>(tab64.size() * 4, 1));
  const size_t o_wa = cur; cur = align_up(cur + std::max<size_t>(h->work_a.size(), 1) * sizeof(int4));
  const size_t o_wb = cur; cur = align_up(cur + work_b.size() * sizeof(int4));
  const size_t o_wl = cur; cur = align_up(cur + std::max<size_t>(h->work_l.size(), 1) * sizeof(int4));
  const size_t o_part = cur; cur = align_up(cur + (size_t)kMaxDots * kRedBlocks * 8);
  const size_t o_S = cur; cur = align_up(cur + kScal * 8);
  const size_t o_map = cur; cur = align_up(cur + (2 * (size_t)kRedBlocks + 1 + n_domains) * sizeof(SegDev));
  const size_t sd_bytes = (size_t)n_domains * (kSD + 1) * 8 + (size_t)n_domains * 4;
  const size_t o_SD = cur; cur = align_up(cur + sd_bytes);
  const size_t o_learn = cur;
  if (h->use_learned) cur = align_up(cur + fmp_coarse_workspace(h->nsub, 512));
  const size_t o_ib = cur;
  if (h->ib.on) cur = align_up(cur + ib_workspace_bytes(h.get()));
  // staging buffers: one per batch stream (a tunable handle keeps room for
  // the most streams fmp_autotune tries)
  h->n_wbuf = h->tunable ? fmp_ctx::kMaxStreams : (h->launches.size() > 1 ? 2 : 1);
  const size_t o_W = cur;
  cur = align_up(cur + (size_t)h->n_wbuf * align_up((size_t)w_batch_max * wsz));
  const size_t need = cur;

  if (!ws) {
    *ws_bytes = need;
    return FMP_OK;
  }
  // The library is built against one HIP release and runs on whichever
  // libamdhip64 the process loaded first (a framework may bundle its own).
  // A different major release changes the runtime ABI: refuse it here rather
  // than fail somewhere inside a launch.
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) != hipSuccess || rt / 10000000 != HIP_VERSION_MAJOR) {
    h->err = "HIP runtime " + std::to_string(rt) + " does not match the major release of the "
             "headers the library was built with (" + std::to_string(HIP_VERSION) + ")";
    return FMP_ERR_UNSUPPORTED;
  }
  if (*ws_bytes < need) return FMP_ERR_WORKSPACE;
  if (((uintptr_t)ws) % kAlign) return FMP_ERR_WORKSPACE;
  if (!out) return FMP_ERR_INVALID_ARG;
  char* base = (char*)ws;
  h->d_doms = (DomainDev*)(base + o_doms);
  h->d_boxes = (BoxDev*)(base + o_boxes);
  for (int v = 0; v < kNumStencilTY; ++v) h->d_tiles_v[v] = (StencilTile*)(base + o_tiles) + tile0[v];
  h->d_tiles = h->d_tiles_v[h->stencil_v];
  h->d_eps = (double*)(base + o_eps);
  h->d_tab = base + o_tab;
  h->d_sig32 = (float*)(base + o_sig32);
  h->d_work_a = (int4*)(base + o_wa);
  h->d_work_b = (int4*)(base + o_wb);
  h->d_work_l = (int4*)(base + o_wl);
  h->d_part = (double*)(base + o_part);
  h->d_S = (double*)(base + o_S);
  h->d_map_glob = (SegDev*)(base + o_map);
  h->d_map_dom = h->d_map_glob + kRedBlocks;
  h->d_segs_glob = h->d_map_dom + kRedBlocks;
  h->d_segs_dom = h->d_segs_glob + 1;
  h->d_SD = (double*)(base + o_SD);
  h->d_fac = h->d_SD + (size_t)n_domains * kSD;
  h->d_act = (int*)(h->d_fac + n_domains);
  for (int i = 0; i < h->n_wbuf; ++i)
    h->d_Wk[i] = base + o_W + (size_t)i * align_up((size_t)w_batch_max * wsz);
  h->d_W = h->d_Wk[0];
  if (h->use_learned) fmp_coarse_bind(h.get(), base + o_learn);

  // typed tables
  std::vector<char> tabbytes(tab_bytes);
  std::vector<float> sig32(tab64.size());
  for (size_t i = 0; i < tab64.size(); ++i) {
    sig32[i] = (float)tab64[i];
    if (h->prec == FMP_FP64) memcpy(&tabbytes[i * 8], &tab64[i], 8);
    else if (h->prec == FMP_FP32) { float f = (float)tab64[i]; memcpy(&tabbytes[i * 4], &f, 4); }
  }
  if (h->prec == FMP_BF16 && tab_bytes) memcpy(tabbytes.data(), tab16.data(), tab_bytes);
  hipStream_t s = (hipStream_t)stream;
  fmp_ctx* hp = h.get();
  HIPCHK(hp, hipMemcpyAsync(h->d_doms, h->doms.data(), h->doms.size() * sizeof(DomainDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_boxes, h->boxes.data(), h->boxes.size() * sizeof(BoxDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_tiles_v[0], tiles.data(), tiles.size() * sizeof(StencilTile),
                            hipMemcpyHostToDevice, s));
  if (!eps_all.empty())
    HIPCHK(hp, hipMemcpyAsync(h->d_eps, eps_all.data(), eps_all.size() * 8, hipMemcpyHostToDevice, s));
  if (!tabbytes.empty())
    HIPCHK(hp, hipMemcpyAsync(h->d_tab, tabbytes.data(), tabbytes.size(), hipMemcpyHostToDevice, s));
  if (!sig32.empty())
    HIPCHK(hp, hipMemcpyAsync(h->d_sig32, sig32.data(), sig32.size() * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_work_a, h->work_a.data(), h->work_a.size() * sizeof(int4),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_work_b, work_b.data(), work_b.size() * sizeof(int4),
                            hipMemcpyHostToDevice, s));
  if (!h->work_l.empty())
    HIPCHK(hp, hipMemcpyAsync(h->d_work_l, h->work_l.data(), h->work_l.size() * sizeof(int4),
                              hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_map_glob, map_glob.data(), kRedBlocks * sizeof(SegDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_map_dom, map_dom.data(), kRedBlocks * sizeof(SegDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_segs_glob, map_glob.data(), sizeof(SegDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipMemcpyAsync(h->d_segs_dom, segs_dom.data(), n_domains * sizeof(SegDev),
                            hipMemcpyHostToDevice, s));
  HIPCHK(hp, hipHostMalloc((void**)&h->h_S, kScal * 8, hipHostMallocDefault));
  HIPCHK(hp, hipHostMalloc((void**)&h->h_SD, sd_bytes, hipHostMallocDefault));
  h->h_fac = h->h_SD + (size_t)n_domains * kSD;
  h->h_act = (int*)(h->h_fac + n_domains);
  HIPCHK(hp, hipStreamSynchronize(s));   // host staging vectors go out of scope
  if (h->ib.on) {
    const fmp_status st = ib_bind(hp, base + o_ib, s);
    if (st != FMP_OK) return st;
  }
  *out = h.release();
  return FMP_OK;
}

fmp_status fmp_vector_layout(fmp_handle h, int64_t* offsets) {
  if (!h || !offsets) return FMP_ERR_INVALID_ARG;
  for (size_t i = 0; i < h->offsets.size(); ++i) offsets[i] = h->offsets[i];
  return FMP_OK;
}

fmp_status fmp_destroy(fmp_handle h) {
  if (!h) return FMP_ERR_INVALID_ARG;
  // Graph replays of this handle may still run on any stream a caller passed;
  // every executable graph, private stream, event and pinned mirror is
  // released only once the device has drained them.
  const hipError_t sync = hipDeviceSynchronize();
  for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
  h->graphs.clear();
  if (h->h_S) (void)hipHostFree(h->h_S);
  if (h->h_SD) (void)hipHostFree(h->h_SD);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (int i = 0; i < fmp_ctx::kMaxStreams; ++i) {
    if (h->bat_stream[i]) (void)hipStreamDestroy(h->bat_stream[i]);
    if (h->ev_join[i]) (void)hipEventDestroy(h->ev_join[i]);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  delete h;
  return sync == hipSuccess ? FMP_OK : FMP_ERR_HIP;
}

fmp_status fmp_curlcurl_apply(fmp_handle h, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return FMP_ERR_INVALID_ARG;
  if (overlaps(x, y, h->len * 8)) return FMP_ERR_ALIAS;
  return spmv(h, x, y, (hipStream_t)stream);
}

fmp_status fmp_apply_precond(fmp_handle h, const double* r, double* z, void* stream) {
  if (!h || !r || !z) return FMP_ERR_INVALID_ARG;
  if (overlaps(r, z, h->len * 8)) return FMP_ERR_ALIAS;
  if (!h->precond_ok) {
    h->err = "a box side exceeds the largest compiled transform size (96 cells for PEC boxes, 48 for index blocks)";
    return FMP_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  const double* coarse = nullptr;
  if (h->learned_set) {
    fmp_status st = fmp_coarse_forward(h, r, s, &coarse);
    if (st != FMP_OK) return st;
  }
  return precond_apply(h, r, z, s, coarse);
}

fmp_status fmp_autotune(fmp_handle h, const double* r, double* z, fmp_tune_entry* entries,
                        int32_t max_entries, int32_t* n_entries, void* stream) {
  if (!h || !r || !z || max_entries < 0) return FMP_ERR_INVALID_ARG;
  if (overlaps(r, z, h->len * 8)) return FMP_ERR_ALIAS;
  if (!h->precond_ok) return FMP_ERR_UNSUPPORTED;
  if (!h->tunable) {
    h->err = "fmp_autotune needs a handle set up with batch_boxes = -1";
    return FMP_ERR_UNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  const int nbox = (int)h->boxes.size();
  std::vector<int> batches;
  for (int b : {16, 32, 64, 128, 256, 512, 1024})
    if (b < nbox) batches.push_back(b);
  batches.push_back(nbox);
  struct Cand { int batch, ns, slab, ty; double ms; };   // ty > 0: a stencil candidate
  std::vector<Cand> cands;
  for (int b : batches)
    for (int ns = 1; ns <= std::min(h->n_wbuf, fmp_ctx::kMaxStreams); ++ns)
      for (int so = 0; so < 2; ++so) cands.push_back({b, ns, so, 0, 0.0});
  for (int v = 0; v < kNumStencilTY; ++v) cands.push_back({0, 0, 0, kStencilTYs[v], 0.0});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const double* coarse = nullptr;   // the learned part does not depend on the plan
  auto use = [&](int b, int ns, int so) -> fmp_status {
    // a captured apply may still be replaying on some caller stream: drain
    // the device before its executable graph is released
    if (!h->graphs.empty()) {
      HIPCHK(h, hipDeviceSynchronize());
      for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
      h->graphs.clear();
    }
    h->slab_order = so;
    plan_batches(h, b);
    h->nstreams = ns;
    HIPCHK(h, hipMemcpyAsync(h->d_boxes, h->boxes.data(), h->boxes.size() * sizeof(BoxDev),
                             hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_work_a, h->work_a.data(), h->work_a.size() * sizeof(int4),
                             hipMemcpyHostToDevice, s));
    if (!h->work_l.empty())
      HIPCHK(h, hipMemcpyAsync(h->d_work_l, h->work_l.data(), h->work_l.size() * sizeof(int4),
                               hipMemcpyHostToDevice, s));
    HIPCHK(h, hipStreamSynchronize(s));
    return FMP_OK;
  };
  auto use_stencil = [&](int ty) {
    for (int v = 0; v < kNumStencilTY; ++v)
      if (kStencilTYs[v] == ty) h->stencil_v = v;
    h->d_tiles = h->d_tiles_v[h->stencil_v];
    h->ntiles = h->ntiles_v[h->stencil_v];
  };
  // mean time of `reps` runs of fn after one warm-up
  auto time_of = [&](auto fn, int reps, double* ms_out) -> fmp_status {
    fmp_status st = fn();
    if (st != FMP_OK) return st;
    HIPCHK(h, hipEventRecord(e0, s));
    for (int k = 0; k < reps && st == FMP_OK; ++k) st = fn();
    if (st != FMP_OK) return st;
    HIPCHK(h, hipEventRecord(e1, s));
    HIPCHK(h, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / reps;
    return FMP_OK;
  };
  auto apply_once = [&]() { return precond_launches(h, r, z, s, coarse); };
  auto spmv_once = [&]() { return spmv(h, r, z, s); };

  // persistent plan cache: FMP_TUNE_CACHE names a text file of
  // "key batch streams slab_order stencil_ty" lines
  const std::string key = tune_key(h);
  const char* cache_path = getenv("FMP_TUNE_CACHE");
  Cand hit{0, 0, 0, 0, -1.0};
  bool cached = false;
  if (cache_path && *cache_path) cached = tune_cache_find(cache_path, key, &hit.batch, &hit.ns,
                                                           &hit.slab, &hit.ty);
  fmp_status st = FMP_OK;
  const Cand* best = nullptr;
  const Cand* best_st = nullptr;
  if (cached) {
    cands.assign({Cand{hit.batch, hit.ns, hit.slab, 0, 0.0}, Cand{0, 0, 0, hit.ty, 0.0}});
    best = &cands[0];
    best_st = &cands[1];
  }
  for (Cand& c : cands) {
    if (c.ty > 0) {                               // stencil tile height
      use_stencil(c.ty);
      if ((st = time_of(spmv_once, 5, &c.ms)) != FMP_OK) break;
      continue;
    }
    if ((st = use(c.batch, c.ns, c.slab)) != FMP_OK) break;
    if (c.ns > 1 && (int)h->launches.size() < c.ns) { c.ms = -1.0; continue; }   // no more overlap
    // candidates are timed as plain launch sequences (no capture per
    // candidate); a graph-mode handle captures the chosen plan on first use
    if ((st = time_of(apply_once, 3, &c.ms)) != FMP_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FMP_OK) return st;
  if (!cached) {
    for (const Cand& c : cands) {
      if (c.ms < 0.0) continue;
      if (c.ty == 0 && (!best || c.ms < best->ms)) best = &c;
      if (c.ty > 0 && (!best_st || c.ms < best_st->ms)) best_st = &c;
    }
  }
  if (!best || !best_st) {
    h->err = "fmp_autotune: no plan could be timed";
    return FMP_ERR_UNSUPPORTED;
  }
  if ((st = use(best->batch, best->ns, best->slab)) != FMP_OK) return st;
  use_stencil(best_st->ty);
  if (!cached && cache_path && *cache_path)
    tune_cache_add(cache_path, key, best->batch, best->ns, best->slab, best_st->ty);
  int k = 0;
  for (const Cand& c : cands) {
    if (c.ms < 0.0) continue;
    if (entries && k < max_entries)
      entries[k] = fmp_tune_entry{c.batch, c.ns, c.slab, c.ms, (&c == best || &c == best_st),
                                  c.ty, cached ? 1 : 0};
    ++k;
  }
  if (n_entries) *n_entries = std::min(k, max_entries);
  return FMP_OK;
}

fmp_status fmp_solve_workspace(fmp_handle h, const fmp_solve_opts* o, size_t* bytes) {
  if (!h || !o || !bytes) return FMP_ERR_INVALID_ARG;
  const size_t vb = align_up((size_t)h->len * 8);
  if (o->solver == 0) *bytes = 8 * vb;
  else if (o->solver == 1) {
    if (o->restart < 1 || o->restart > 32) return FMP_ERR_INVALID_ARG;
    *bytes = (2 * (size_t)o->restart + 1) * vb;
  } else return FMP_ERR_INVALID_ARG;
  return FMP_OK;
}

}  // extern "C"

// ============================================================== solvers
namespace {

// Event timing of kernel classes for opts.profile.  Pairs are recorded
// around launches and read back at the solver's next synchronisation.
struct Prof {
  enum { PRE = 0, SPMV = 1, DOT = 2, UPD = 3 };
  std::vector<hipEvent_t> pool;
  struct Pending {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Pending> pend;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Prof() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct Ctx {
  fmp_ctx* h;
  hipStream_t s;
  const fmp_solve_opts* o;
  fmp_solve_info* info;
  Prof* prof;
  // bracket a launch sequence with events when profiling
  hipEvent_t begin() {
    if (!prof) return nullptr;
    hipEvent_t e = prof->get();
    if (e) (void)hipEventRecord(e, s);
    return e;
  }
  void end(int cls, hipEvent_t a) {
    if (!prof || !a) return;
    hipEvent_t b = prof->get();
    if (!b) return;
    (void)hipEventRecord(b, s);
    prof->pend.push_back({cls, a, b});
  }
  // after a synchronisation: accumulate the recorded pairs
  void harvest() {
    if (!prof) return;
    for (const auto& p : prof->pend) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) continue;
      double* t = p.cls == Prof::PRE    ? &info->t_precond_ms
                  : p.cls == Prof::SPMV ? &info->t_spmv_ms
                  : p.cls == Prof::DOT  ? &info->t_orth_dot_ms
                                        : &info->t_orth_update_ms;
      *t += ms;
    }
    prof->pend.clear();
    prof->used = 0;
  }
};

// z = M^{-1} r; the learned coarse correction is added only where the caller
// can test it (FGMRES), since BiCGSTAB assumes a fixed linear preconditioner.
fmp_status M_(Ctx& c, const double* r, double* z, bool learned);
fmp_status M(Ctx& c, const double* r, double* z, bool learned = false) {
  hipEvent_t e = c.begin();
  const fmp_status st = M_(c, r, z, learned);
  c.end(Prof::PRE, e);
  return st;
}
fmp_status M_(Ctx& c, const double* r, double* z, bool learned) {
  c.info->n_precond++;
  if (c.o->precond == 0) {
    HIPCHK(c.h, launch_scale_copy(r, 1.0, z, c.h->len, c.s));
    return FMP_OK;
  }
  const double* coarse = nullptr;
  if (learned && c.h->learned_set) {
    fmp_status st = fmp_coarse_forward(c.h, r, c.s, &coarse);
    if (st != FMP_OK) return st;
  }
  return precond_apply(c.h, r, z, c.s, coarse);
}

fmp_status A(Ctx& c, const double* x, double* y) {
  c.info->n_spmv++;
  hipEvent_t e = c.begin();
  const fmp_status st = spmv(c.h, x, y, c.s);
  c.end(Prof::SPMV, e);
  return st;
}

// Reduction groups of a solve: the whole system (one group), or one group
// per domain (independent solves advanced in lockstep).
struct Groups {
  int n;
  const SegDev* map;    // per block
  const SegDev* segs;   // per group
};

// profiled CGS kernels: h = V^T w (+ ||w||^2), then w -= V h (+ ||w||^2);
// act_len = elements of the groups taking part (for the byte count)
hipError_t orth_dot(Ctx& c, const Groups& G, const int* act, double act_len, const double* V,
                    long long ldv, int nv, const double* w) {
  hipEvent_t e = c.begin();
  const hipError_t r = launch_mdot(V, ldv, nv, w, G.map, act, c.h->d_part, c.s);
  c.end(Prof::DOT, e);
  c.info->n_orth_dot++;
  c.info->bytes_orth_dot += 8.0 * act_len * (nv + 1);
  return r;
}
hipError_t orth_update(Ctx& c, const Groups& G, const int* act, double act_len, const double* V,
                       long long ldv, int nv, const double* hcoef, const double* sc, int hld,
                       double* w) {
  hipEvent_t e = c.begin();
  const hipError_t r =
      launch_mupdate(V, ldv, nv, hcoef, sc, hld, w, G.map, act, c.h->d_part, c.s);
  c.end(Prof::UPD, e);
  c.info->n_orth_update++;
  c.info->bytes_orth_update += 8.0 * act_len * (nv + 2);
  return r;
}

// r = b - A x with wall slots 0 (tmp holds A x); ||r_d||^2 per domain into
// rr[0..ndom) (host), summed in domain order into *total.
fmp_status residual(Ctx& c, const double* b, const double* x, double* r, double* tmp,
                    std::vector<double>& rr, double* total) {
  fmp_status st = A(c, x, tmp);
  if (st) return st;
  fmp_ctx* h = c.h;
  const int nd = (int)h->doms.size();
  HIPCHK(h, launch_sub_norm(b, tmp, r, h->d_map_dom, h->d_doms, h->d_part, c.s));
  HIPCHK(h, launch_reduce_seg(h->d_part, 1, h->d_segs_dom, nd, h->d_SD + kSDR, kSD, c.s));
  HIPCHK(h, hipMemcpyAsync(h->h_SD, h->d_SD, (size_t)nd * kSD * 8, hipMemcpyDeviceToHost, c.s));
  HIPCHK(h, hipStreamSynchronize(c.s));
  rr.assign(nd, 0.0);
  double t = 0.0;
  for (int d = 0; d < nd; ++d) {
    rr[d] = h->h_SD[(size_t)d * kSD + kSDR];
    t += rr[d];
  }
  *total = t;
  return FMP_OK;
}

// per-domain outputs of a solve
void report_domains(Ctx& c, const std::vector<double>& rr0, const std::vector<double>& rr,
                    const std::vector<int>& iters) {
  const int nd = (int)rr.size();
  for (int d = 0; d < nd; ++d) {
    if (c.o->domain_rel_residual)
      c.o->domain_rel_residual[d] = rr0[d] > 0.0 ? sqrt(rr[d] / rr0[d]) : 0.0;
    if (c.o->domain_iterations) c.o->domain_iterations[d] = iters[d];
  }
}

fmp_status bicgstab(Ctx& c, const double* b, double* x, double* ws) {
  fmp_ctx* h = c.h;
  const long long n = h->len;
  const size_t vb = align_up((size_t)n * 8) / 8;
  double *r = ws, *rhat = ws + vb, *p = ws + 2 * vb, *v = ws + 3 * vb, *phat = ws + 4 * vb,
         *sv = ws + 5 * vb, *shat = ws + 6 * vb, *t = ws + 7 * vb;
  const double tol = c.o->rtol;
  const int check = std::max(1, c.o->check_every);
  double rr;
  std::vector<double> rrd0, rrd;
  HIPCHK(h, launch_zero_walls(x, h->d_doms, (int)h->doms.size(), c.s));
  fmp_status st = residual(c, b, x, r, t, rrd0, &rr);
  if (st) return st;
  if (!isfinite(rr)) return FMP_ERR_BREAKDOWN;
  const double r0 = sqrt(rr);
  c.info->rel_residual_true = 0.0;
  rrd = rrd0;
  auto report = [&](int iters) {
    report_domains(c, rrd0, rrd, std::vector<int>(rrd0.size(), iters));
  };
  if (r0 == 0.0) { report(0); return FMP_OK; }
  int it = 0;
  bool broke = false;
  while (it < c.o->max_iter) {
    HIPCHK(h, hipMemcpyAsync(rhat, r, n * 8, hipMemcpyDeviceToDevice, c.s));
    HIPCHK(h, hipMemsetAsync(p, 0, n * 8, c.s));
    HIPCHK(h, hipMemsetAsync(v, 0, n * 8, c.s));
    double* hs = h->h_S;
    hs[0] = rr; hs[1] = 1.0; hs[2] = 1.0; hs[3] = 1.0; hs[8] = 0.0;
    HIPCHK(h, hipMemcpyAsync(h->d_S, hs, 9 * 8, hipMemcpyHostToDevice, c.s));
    bool restart = false;
    while (it < c.o->max_iter) {
      HIPCHK(h, launch_bicg_p(r, p, v, h->d_S, n, c.s));
      if ((st = M(c, p, phat))) return st;
      if ((st = A(c, phat, v))) return st;
      DotPtrs d1{};
      d1.a[0] = rhat; d1.b[0] = v;
      HIPCHK(h, launch_dots(d1, 1, n, h->d_part, c.s));
      HIPCHK(h, launch_reduce(h->d_part, 1, h->d_S + 4, 1, h->d_S, c.s));
      HIPCHK(h, launch_bicg_s(r, v, sv, h->d_S, n, c.s));
      if ((st = M(c, sv, shat))) return st;
      if ((st = A(c, shat, t))) return st;
      DotPtrs d2{};
      d2.a[0] = t; d2.b[0] = sv; d2.a[1] = t; d2.b[1] = t;
      HIPCHK(h, launch_dots(d2, 2, n, h->d_part, c.s));
      HIPCHK(h, launch_reduce(h->d_part, 2, h->d_S + 5, 2, h->d_S, c.s));
      HIPCHK(h, launch_bicg_xr(x, phat, shat, sv, t, r, rhat, h->d_S, n, h->d_part, c.s));
      HIPCHK(h, launch_reduce(h->d_part, 2, h->d_S + 7, 3, h->d_S, c.s));
      ++it;
      if (it % check == 0 || it >= c.o->max_iter) {
        HIPCHK(h, hipMemcpyAsync(hs, h->d_S, 9 * 8, hipMemcpyDeviceToHost, c.s));
        HIPCHK(h, hipStreamSynchronize(c.s));
        const double rn = sqrt(hs[7]);
        if (!isfinite(rn) || !isfinite(hs[0])) { broke = true; break; }
        if (rn <= tol * r0) { restart = true; break; }
        if (hs[3] == 0.0 || hs[0] == 0.0) { broke = true; break; }
      }
    }
    if ((st = residual(c, b, x, r, t, rrd, &rr))) return st;
    c.info->rel_residual_true = sqrt(rr) / r0;
    if (!isfinite(rr)) broke = true;
    if (!broke && sqrt(rr) <= tol * r0) {
      c.info->iterations = it;
      report(it);
      return FMP_OK;
    }
    if (broke || !restart) break;
  }
  c.info->iterations = it;
  report(it);
  return broke ? FMP_ERR_BREAKDOWN : FMP_NOT_CONVERGED;
}

// Arnoldi state of one group's FGMRES cycle.  The basis is stored
// unnormalised: v_i = s_i V_i, so no pass over the vector is spent on scaling;
// the scales enter the coefficients instead (true h_ij = s_i s_j <V_i, W>,
// update coefficients s_i^2 <V_i, W>, x update coefficients y_i s_i).
struct Arnoldi {
  int m = 0;
  std::vector<double> H, cs, sn, g, y, s;
  double r0 = 0.0, beta = 0.0;
  int ncols = 0;
  bool active = false;     // iterating in the current cycle
  bool finished = false;   // recomputed residual met the tolerance
  int iters = 0;           // Arnoldi steps this group has taken
  void start(int m_, double beta_) {
    m = m_;
    H.assign((size_t)(m + 1) * m, 0.0);
    cs.assign(m, 0.0); sn.assign(m, 0.0); y.assign(m, 0.0);
    g.assign(m + 1, 0.0);
    s.assign(m + 1, 0.0);
    g[0] = beta_;
    s[0] = beta_ > 0.0 ? 1.0 / beta_ : 0.0;
    ncols = 0;
  }
  // append column j (h_0..h_j, h_{j+1} = hn), rotate it, return |g_{j+1}|
  double add(int j, const double* hcol, double hn) {
    for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i];
    H[(j + 1) * m + j] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = H[i * m + j], bb = H[(i + 1) * m + j];
      H[i * m + j] = cs[i] * a + sn[i] * bb;
      H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
    }
    const double a = H[j * m + j], bb = H[(j + 1) * m + j];
    const double den = hypot(a, bb);
    cs[j] = den == 0.0 ? 1.0 : a / den;
    sn[j] = den == 0.0 ? 0.0 : bb / den;
    H[j * m + j] = cs[j] * a + sn[j] * bb;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    ncols = j + 1;
    return fabs(g[j + 1]);
  }
  // back substitution of the triangular least-squares system
  void solve() {
    for (int i = ncols - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < ncols; ++k) acc -= H[i * m + k] * y[k];
      y[i] = acc / H[i * m + i];
    }
  }
};

fmp_status fgmres(Ctx& c, const double* b, double* x, double* ws) {
  fmp_ctx* h = c.h;
  const long long n = h->len;
  const int m = c.o->restart;
  const size_t vb = align_up((size_t)n * 8) / 8;
  double* V = ws;
  double* Z = ws + (size_t)(m + 1) * vb;
  const double tol = c.o->rtol;
  const int nd = (int)h->doms.size();
  const bool per = c.o->per_domain && nd > 1;
  const Groups G = per ? Groups{nd, h->d_map_dom, h->d_segs_dom}
                       : Groups{1, h->d_map_glob, h->d_segs_glob};
  const int ng = G.n;
  double* hs = h->h_S;
  double* SD = h->h_SD;
  std::vector<Arnoldi> grp(ng);
  std::vector<double> glen(ng, 0.0);
  for (int d = 0; d < nd; ++d) glen[per ? d : 0] += (double)h->seg_len[d];

  HIPCHK(h, launch_zero_walls(x, h->d_doms, nd, c.s));
  std::vector<double> rrd0, rrd;
  double tot;
  fmp_status st = residual(c, b, x, V, Z, rrd0, &tot);
  if (st) return st;
  rrd = rrd0;
  std::vector<int> dom_it(nd, 0);
  auto group_rr = [&](const std::vector<double>& rr, int g) {
    if (per) return rr[g];
    double t = 0.0;
    for (double v : rr) t += v;
    return t;
  };
  auto finish = [&](int it, fmp_status code) {
    c.info->iterations = it;
    double worst = 0.0;
    for (int g = 0; g < ng; ++g)
      worst = std::max(worst, grp[g].r0 > 0.0 ? grp[g].beta / grp[g].r0 : 0.0);
    c.info->rel_residual_true = worst;
    for (int d = 0; d < nd; ++d) dom_it[d] = per ? grp[d].iters : it;
    report_domains(c, rrd0, rrd, dom_it);
    return code;
  };
  bool all_done = true;
  for (int g = 0; g < ng; ++g) {
    const double r2 = group_rr(rrd0, g);
    if (!isfinite(r2)) return FMP_ERR_BREAKDOWN;
    grp[g].r0 = grp[g].beta = sqrt(r2);
    grp[g].finished = grp[g].r0 == 0.0;
    all_done = all_done && grp[g].finished;
  }
  if (all_done) return finish(0, FMP_OK);

  auto active_len = [&]() {
    double t = 0.0;
    for (int g = 0; g < ng; ++g)
      if (grp[g].active) t += glen[g];
    return t;
  };
  // host scalars (squared basis scales, update coefficients) and activity
  // flags to the device
  int* act = h->h_act;
  auto push = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(h->d_SD, SD, (size_t)ng * kSD * 8, hipMemcpyHostToDevice, c.s);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(h->d_act, act, (size_t)ng * 4, hipMemcpyHostToDevice, c.s);
  };
  // Explicit scaling of a stored basis vector, per group: 0 for groups that
  // stopped while others go on (their part of later vectors stays 0), s for
  // groups whose stored norm 1/s left [1e-15, 1e15] (the reduced-precision
  // transforms must not see under- or overflowing inputs), 1 (skipped) else.
  auto fix_scale = [&](double* v, const std::vector<double>& fac) -> fmp_status {
    bool any = false;
    for (int g = 0; g < ng; ++g) {
      h->h_fac[g] = fac[g];
      any = any || fac[g] != 1.0;
    }
    if (!any) return FMP_OK;
    HIPCHK(h, hipMemcpyAsync(h->d_fac, h->h_fac, (size_t)ng * 8, hipMemcpyHostToDevice, c.s));
    HIPCHK(h, launch_scale_seg(v, h->d_fac, v, G.map, c.s));
    return FMP_OK;
  };

  // the learned part stays on while the FP64 residual test keeps accepting
  // it; after kMaxRejects rejections in a row the solve continues without it
  constexpr int kMaxRejects = 3;
  bool use_learned = !per && c.o->precond != 0 && h->learned_set;
  int rejects = 0;
  int it = 0;
  while (it < c.o->max_iter) {
    // new cycle: V_0 = r (stored unnormalised, s_0 = 1 / beta); finished
    // groups get V_0 = 0
    std::vector<double> fac(ng, 1.0);
    for (int g = 0; g < ng; ++g) {
      Arnoldi& A_ = grp[g];
      A_.active = !A_.finished;
      A_.start(m, A_.active ? A_.beta : 0.0);
      if (!A_.active) fac[g] = 0.0;
      else if (A_.s[0] > 1e15 || A_.s[0] < 1e-15) { fac[g] = A_.s[0]; A_.s[0] = 1.0; }
      SD[(size_t)g * kSD + kSDS] = A_.s[0] * A_.s[0];
      act[g] = A_.active ? 1 : 0;
    }
    HIPCHK(h, push());
    if ((st = fix_scale(V, fac))) return st;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (size_t)j * vb;
      double* zj = Z + (size_t)j * vb;
      double* w = V + (size_t)(j + 1) * vb;
      const bool learned = use_learned;
      if ((st = M(c, vj, zj, learned))) return st;
      if ((st = A(c, zj, w))) return st;
      if (learned) {
        // the FP64 residual decides on the correction: keep it only if
        // ||v - A z|| does not exceed the plain preconditioner's ||v - A z_RAS||
        // (both sides carry the same basis scale)
        HIPCHK(h, fmp_coarse_resid_test(h, vj, w, h->d_part, c.s));
        HIPCHK(h, launch_reduce(h->d_part, 2, h->d_S + kScalJ, 0, h->d_S, c.s));
        HIPCHK(h, hipMemcpyAsync(hs + kScalJ, h->d_S + kScalJ, 16, hipMemcpyDeviceToHost, c.s));
        HIPCHK(h, hipStreamSynchronize(c.s));
        if (!(hs[kScalJ] <= hs[kScalJ + 1])) {
          c.info->used_fallback++;
          c.info->n_precond++;
          if ((st = precond_apply(h, vj, zj, c.s, nullptr))) return st;
          if ((st = A(c, zj, w))) return st;
          if (++rejects >= kMaxRejects) use_learned = false;
        } else {
          rejects = 0;
        }
      }
      // classical Gram-Schmidt per group on the stored vectors:
      // h~ = V^T W (and ||W||^2), W -= V (s^2 h~), ||W||^2
      const double alen = active_len();
      HIPCHK(h, orth_dot(c, G, h->d_act, alen, V, (long long)vb, j + 1, w));
      HIPCHK(h, launch_reduce_seg(h->d_part, j + 2, G.segs, ng, h->d_SD + kSDH, kSD, c.s));
      HIPCHK(h, orth_update(c, G, h->d_act, alen, V, (long long)vb, j + 1, h->d_SD + kSDH,
                            h->d_SD + kSDS, kSD, w));
      HIPCHK(h, launch_reduce_seg(h->d_part, 1, G.segs, ng, h->d_SD + kSDW, kSD, c.s));
      HIPCHK(h, hipMemcpyAsync(SD, h->d_SD, (size_t)ng * kSD * 8, hipMemcpyDeviceToHost, c.s));
      HIPCHK(h, hipStreamSynchronize(c.s));
      c.harvest();
      // true coefficients: h_ij = s_i s_j h~_i, ||w|| = s_j ||W||
      std::vector<double> hcol((size_t)ng * (j + 1)), wn(ng, 0.0);
      bool reorth = false;
      for (int g = 0; g < ng; ++g) {
        act[g] = 0;
        if (!grp[g].active) continue;
        const Arnoldi& A_ = grp[g];
        const double* sg = SD + (size_t)g * kSD;
        for (int i = 0; i <= j; ++i)
          hcol[(size_t)g * (j + 1) + i] = A_.s[i] * A_.s[j] * sg[kSDH + i];
        const double wn0 = sqrt(sg[kSDH + j + 1]);
        wn[g] = sqrt(sg[kSDW]);
        if (wn[g] < 0.1 * wn0) { act[g] = 1; reorth = true; }   // second CGS pass
      }
      if (reorth) {
        double rlen = 0.0;
        for (int g = 0; g < ng; ++g)
          if (act[g]) rlen += glen[g];
        HIPCHK(h, hipMemcpyAsync(h->d_act, act, (size_t)ng * 4, hipMemcpyHostToDevice, c.s));
        HIPCHK(h, orth_dot(c, G, h->d_act, rlen, V, (long long)vb, j + 1, w));
        HIPCHK(h, launch_reduce_seg(h->d_part, j + 2, G.segs, ng, h->d_SD + kSDH, kSD, c.s));
        HIPCHK(h, orth_update(c, G, h->d_act, rlen, V, (long long)vb, j + 1, h->d_SD + kSDH,
                              h->d_SD + kSDS, kSD, w));
        HIPCHK(h, launch_reduce_seg(h->d_part, 1, G.segs, ng, h->d_SD + kSDW, kSD, c.s));
        HIPCHK(h, hipMemcpyAsync(SD, h->d_SD, (size_t)ng * kSD * 8, hipMemcpyDeviceToHost, c.s));
        HIPCHK(h, hipStreamSynchronize(c.s));
        c.harvest();
        for (int g = 0; g < ng; ++g) {
          if (!act[g]) continue;
          const Arnoldi& A_ = grp[g];
          const double* sg = SD + (size_t)g * kSD;
          for (int i = 0; i <= j; ++i)
            hcol[(size_t)g * (j + 1) + i] += A_.s[i] * A_.s[j] * sg[kSDH + i];
          wn[g] = sqrt(sg[kSDW]);
        }
      }
      ++it;
      bool any = false;
      std::fill(fac.begin(), fac.end(), 1.0);
      for (int g = 0; g < ng; ++g) {
        Arnoldi& A_ = grp[g];
        act[g] = 0;
        if (!A_.active) continue;
        const double hn = A_.s[j] * wn[g];
        if (!isfinite(hn)) return FMP_ERR_BREAKDOWN;
        const double est = A_.add(j, &hcol[(size_t)g * (j + 1)], hn);
        A_.iters++;
        if (hn == 0.0 || est <= tol * A_.r0) {
          A_.active = false;
          fac[g] = 0.0;
        }
        any = any || A_.active;
        A_.s[j + 1] = A_.active ? 1.0 / wn[g] : 0.0;    // v_{j+1} = W / ||W||
        if (A_.active && (A_.s[j + 1] > 1e15 || A_.s[j + 1] < 1e-15)) {
          fac[g] = A_.s[j + 1];
          A_.s[j + 1] = 1.0;
        }
        SD[(size_t)g * kSD + kSDS + j + 1] = A_.s[j + 1] * A_.s[j + 1];
        act[g] = A_.active ? 1 : 0;
      }
      if (c.o->capture && it <= c.o->capture_count) {   // x_it = x + Z y (one group)
        Arnoldi& A0 = grp[0];
        A0.solve();
        for (int i = 0; i < A0.ncols; ++i) SD[kSDY + i] = A0.y[i] * A0.s[i];
        double* slot = c.o->capture + (size_t)(it - 1) * n;
        HIPCHK(h, hipMemcpyAsync(h->d_SD + kSDY, SD + kSDY, A0.ncols * 8, hipMemcpyHostToDevice, c.s));
        HIPCHK(h, hipMemcpyAsync(slot, x, n * 8, hipMemcpyDeviceToDevice, c.s));
        HIPCHK(h, launch_xupdate(Z, (long long)vb, A0.ncols, h->d_SD + kSDY, kSD, slot, G.map, c.s));
        HIPCHK(h, hipStreamSynchronize(c.s));
      }
      if (!any || it >= c.o->max_iter) break;
      HIPCHK(h, push());
      if ((st = fix_scale(w, fac))) return st;
    }
    // x += Z (y s) per group (0 beyond a group's own column count)
    int ncmax = 0;
    for (int g = 0; g < ng; ++g) {
      Arnoldi& A_ = grp[g];
      double* sy = SD + (size_t)g * kSD + kSDY;
      for (int i = 0; i < m; ++i) sy[i] = 0.0;
      if (A_.finished || A_.ncols == 0) continue;
      A_.solve();
      for (int i = 0; i < A_.ncols; ++i) sy[i] = A_.y[i] * A_.s[i];
      ncmax = std::max(ncmax, A_.ncols);
    }
    if (ncmax > 0) {
      HIPCHK(h, hipMemcpyAsync(h->d_SD, SD, (size_t)ng * kSD * 8, hipMemcpyHostToDevice, c.s));
      HIPCHK(h, launch_xupdate(Z, (long long)vb, ncmax, h->d_SD + kSDY, kSD, x, G.map, c.s));
    }
    if ((st = residual(c, b, x, V, Z, rrd, &tot))) return st;
    all_done = true;
    for (int g = 0; g < ng; ++g) {
      Arnoldi& A_ = grp[g];
      if (A_.finished) continue;
      const double r2 = group_rr(rrd, g);
      if (!isfinite(r2)) return finish(it, FMP_ERR_BREAKDOWN);
      A_.beta = sqrt(r2);
      A_.finished = A_.beta <= tol * A_.r0;
      all_done = all_done && A_.finished;
    }
    if (all_done) return finish(it, FMP_OK);
  }
  return finish(it, FMP_NOT_CONVERGED);
}

}  // namespace

extern "C" fmp_status fmp_solve(fmp_handle h, const double* b, double* x, const fmp_solve_opts* o,
                                void* ws, size_t ws_bytes, fmp_solve_info* info, void* stream) {
  if (!h || !b || !x || !o || !ws) return FMP_ERR_INVALID_ARG;
  if (o->max_iter < 1 || !(o->rtol > 0.0)) return FMP_ERR_INVALID_ARG;
  if (o->capture_count < 0 || (o->capture_count > 0 && (!o->capture || o->solver != 1)))
    return FMP_ERR_INVALID_ARG;
  if (o->per_domain && o->capture_count > 0 && h->doms.size() > 1) return FMP_ERR_INVALID_ARG;
  if (o->per_domain && h->doms.size() > 1 &&
      (o->solver != 1 || (o->precond && h->learned_set))) {
    h->err = "per-domain solves run FGMRES without the learned part";
    return FMP_ERR_UNSUPPORTED;
  }
  if (overlaps(b, x, h->len * 8)) return FMP_ERR_ALIAS;
  size_t need = 0;
  fmp_status st = fmp_solve_workspace(h, o, &need);
  if (st) return st;
  if (ws_bytes < need || ((uintptr_t)ws) % kAlign) return FMP_ERR_WORKSPACE;
  if (o->precond && !h->precond_ok) return FMP_ERR_UNSUPPORTED;
  fmp_solve_info local{};
  Prof prof;
  Ctx c{h, (hipStream_t)stream, o, &local, o->profile ? &prof : nullptr};
  const auto t0 = std::chrono::steady_clock::now();
  st = (o->solver == 0) ? bicgstab(c, b, x, (double*)ws) : fgmres(c, b, x, (double*)ws);
  if (hipStreamSynchronize(c.s) != hipSuccess && st >= 0) st = FMP_ERR_HIP;
  c.harvest();
  local.t_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = local;
  return st;
}
