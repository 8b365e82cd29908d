// Host state of the batched form (grasp_batch_*).
#pragma once

#include <map>
#include <tuple>
#include <vector>

#include "context.h"

namespace grasp {

struct BatchView {
  HandView hand;
  SdfView sdf;
  StepConsts prm;
};

struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

float dilation_at(float r0, int32_t t, int32_t T);

}  // namespace grasp

struct grasp_batch {
  grasp_ctx* ctx = nullptr;
  int32_t capacity = 0;       // most candidates one step may hold
  int32_t max_jobs = 0;
  bool use_graph = true;
  size_t half = 0;            // bytes of one table (header + jobs), 256-aligned
  char* dev = nullptr;        // [K=1 table][K>1 table][per-job non-finite flags][orders]
  char* host = nullptr;       // pinned staging of both tables
  int* flags_dev = nullptr;
  int* order_dev = nullptr;   // per-job candidate locality orders, capacity ints
  grasp::TileCfg tile{};
  std::vector<grasp::BatchView> views;
  std::map<std::tuple<int, int, int, int>, grasp::BatchGraph> graphs;  // (group + 2 fric, wpb, occ, lds)
  hipEvent_t last = nullptr;  // completion of the previous step (table reuse)
};
