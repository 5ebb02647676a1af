// Handle of the FlashMP library (internal; shared by the host-side sources).
#pragma once

#include <string>
#include <vector>

#include "fmp_common.h"

using fmp::BoxDev;
using fmp::DomainDev;
using fmp::StencilTile;
using fmp::IBCorrDev;

struct Launch {
  int cls;
  int a0, na;   // pass A / C work items
  int b0, nb;   // pass B work items
  int l0[3], nl[3];   // large classes (FP64 / FP32): contraction items per axis
};

// Index-block subdomains with Algorithm 1's low-rank boundary correction.
struct IBCorr {
  int nx, ny, nz, wall;   // box shape and low-wall bits
  double alpha;
  int m, mp;              // boundary slots; padded order (multiple of 64)
  int qoff;               // boundary slot list of the shape
  long long off;          // offset (doubles) of C^{-1}
  int rep;                // one box that uses it
};

struct IBPlan {
  bool on = false;
  std::vector<BoxDev> boxes;
  std::vector<double> tab;
  std::vector<int> qidx;
  std::vector<IBCorr> corr;
  struct Cls {
    int np, a0, na, b0, nb;
  };
  std::vector<Cls> cls;
  std::vector<int4> work_a, work_b;
  std::vector<int4> gemv;      // (correction, first row, first gbox entry, boxes)
  std::vector<int> gbox;       // boxes grouped by correction matrix
  long long w_elems = 0;       // staging of all boxes (one buffer)
  long long g_elems = 0;
  long long cinv_elems = 0;
  long long stage_elems = 0;   // W_E + W_C region (also the unit-solve staging at setup)
  int unit_batch = 0;
  int m_max = 0, mp_max = 0;
  int gemv_kr = 1024;          // rows of C^{-1} per k-range of the C^{-1} h step
  long long vol_max = 0;
  BoxDev* d_boxes = nullptr;
  double* d_tab = nullptr;
  int* d_qidx = nullptr;
  IBCorrDev* d_corr = nullptr;
  int4* d_work_a = nullptr;
  int4* d_work_b = nullptr;
  int4* d_gemv = nullptr;
  int* d_gbox = nullptr;
  double* d_WE = nullptr;
  double* d_WC = nullptr;
  double* d_g = nullptr;
  double* d_hv = nullptr;
  double* d_part = nullptr;    // partial sums of the C^{-1} h step
  double* d_cinv = nullptr;
  // setup only: pivot block, row and column panels, W^{-1}, unit-box records
  double* d_P = nullptr;
  double* d_Row = nullptr;
  double* d_Col = nullptr;
  double* d_winv = nullptr;
  BoxDev* d_ubox = nullptr;
  int4* d_uwork_a = nullptr;
  int4* d_uwork_b = nullptr;
};

struct fmp_ctx {
  std::vector<DomainDev> doms;
  std::vector<BoxDev> boxes;
  std::vector<long long> offsets;
  std::vector<Launch> launches;
  // batch planning: boxes in class order, each box's first pass-B work item
  // (one extra entry at the end), the staging capacity per W buffer
  // (elements) and the current plan's knobs
  std::vector<int> order, wb0;
  std::vector<int4> work_a;    // pass A / C items of the current plan (see plan_batches)
  std::vector<int4> work_l;    // contraction items of large FP64 / FP32 boxes
  long long w_cap = 0;
  int batch = 0;               // boxes per batch
  int nstreams = 2;            // 1 = batches in order on the caller's stream
  int slab_order = 1;          // pass A / C items: 1 = slab-major, 0 = box-major
  bool tunable = false;
  int prec = 0;
  int overlap = 1;
  bool precond_ok = true;      // every box side has a compiled transform class
  int nsub = 0;
  long long len = 0;
  int ntiles = 0;                      // stencil tiles of the chosen tile height
  int stencil_v = fmp::kStencilDefault;
  int ntiles_v[fmp::kNumStencilTY] = {};
  StencilTile* d_tiles_v[fmp::kNumStencilTY] = {};
  // device regions inside the workspace
  DomainDev* d_doms = nullptr;
  BoxDev* d_boxes = nullptr;
  StencilTile* d_tiles = nullptr;
  double* d_eps = nullptr;
  void* d_tab = nullptr;
  float* d_sig32 = nullptr;
  int4* d_work_a = nullptr;
  int4* d_work_b = nullptr;
  int4* d_work_l = nullptr;
  void* d_W = nullptr;
  double* d_part = nullptr;
  double* d_S = nullptr;
  // learned coarse correction (layout in fmp_coarse.hip)
  bool use_learned = false;
  bool learned_set = false;
  int hidden = 0;
  double* d_rc = nullptr;      // R0 r, [3][nsub]
  double* d_yc = nullptr;      // correction to inject, [3][nsub]
  double* d_cS = nullptr;      // scalars of the coarse step (norm of R0 r)
  float* d_u = nullptr;        // MLP input (R0 r / ||R0 r||)
  float* d_h1 = nullptr;
  float* d_h2 = nullptr;
  __hip_bfloat16* d_W1 = nullptr;
  __hip_bfloat16* d_W2 = nullptr;
  __hip_bfloat16* d_W3 = nullptr;
  float* d_b1 = nullptr;
  float* d_b2 = nullptr;
  float* d_b3 = nullptr;
  double* h_S = nullptr;       // pinned host mirror of scalars
  // reduction segments: one over the whole vector, one per domain
  fmp::SegDev* d_map_glob = nullptr;   // per block (kRedBlocks)
  fmp::SegDev* d_segs_glob = nullptr;  // 1
  fmp::SegDev* d_map_dom = nullptr;    // per block (kRedBlocks)
  fmp::SegDev* d_segs_dom = nullptr;   // one per domain
  std::vector<long long> seg_len;      // elements per domain segment
  // per-group Krylov scalars (group = the whole system, or one domain):
  // kSD doubles per group, then the group scale factors and activity flags
  double* d_SD = nullptr;
  double* d_fac = nullptr;
  int* d_act = nullptr;
  double* h_SD = nullptr;              // pinned mirror of d_SD, d_fac, d_act
  double* h_fac = nullptr;
  int* h_act = nullptr;
  // captured preconditioner applies, keyed by (r, z, learned part active)
  struct Graph {
    const double* r;
    double* z;
    bool coarse;
    hipGraphExec_t exec;
  };
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  // batch k runs on private stream k % nstreams with staging buffer k % nstreams
  static constexpr int kMaxStreams = 2;
  void* d_Wk[kMaxStreams] = {nullptr, nullptr};
  int n_wbuf = 1;
  hipStream_t bat_stream[kMaxStreams] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kMaxStreams] = {nullptr, nullptr};
  std::vector<Graph> graphs;
  IBPlan ib;
  std::string err;
};

// index-block subdomains (fmp_woodbury.hip)
fmp_status ib_prepare(fmp_ctx* h);                       // plans, tables, slot lists
size_t ib_workspace_bytes(const fmp_ctx* h);
fmp_status ib_bind(fmp_ctx* h, char* base, hipStream_t s);   // upload, build C^{-1}
fmp_status ib_apply(fmp_ctx* h, const double* r, double* z, hipStream_t s);

