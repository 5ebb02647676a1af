// Handle of the FlashMP library (internal; shared by the host-side sources).
#pragma once

#include <string>
#include <vector>

#include "fmp_common.h"

using fmp::BoxDev;
using fmp::DomainDev;
using fmp::StencilTile;

struct Launch {
  int cls;
  int a0, na;   // pass A / C work items
  int b0, nb;   // pass B work items
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
  int ntiles = 0;
  // device regions inside the workspace
  DomainDev* d_doms = nullptr;
  BoxDev* d_boxes = nullptr;
  StencilTile* d_tiles = nullptr;
  double* d_eps = nullptr;
  void* d_tab = nullptr;
  float* d_sig32 = nullptr;
  int4* d_work_a = nullptr;
  int4* d_work_b = nullptr;
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
  std::string err;
};

