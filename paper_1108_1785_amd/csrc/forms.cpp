// Batched form: one classify/aggregate step (with its flag step) captured into
// a HIP graph for replay, and an autotuner that times launch shapes on the
// caller's data.  Both drive only the C-ABI entry points of kernels.hip.
//
// The paper runs one monitoring window per hourly launch (§III.B.1, NetPerf
// Monitoring Thread); here many windows of uneven size go through one
// persistent launch, and the launch sequence is replayed as a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "registry.h"

namespace gnm {
namespace {

int hip_err(hipError_t e, const char *where) {
  set_last_error(std::string(where) + ": " + hipGetErrorString(e));
  return GNM_E_HIP;
}

}  // namespace
}  // namespace gnm

using namespace gnm;

struct gnm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
};

extern "C" int gnm_graph_create(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                                uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint64_t threshold_bps,
                                uint64_t min_bulk_flows, uint8_t *flags, gnm_graph **out) {
  if (!out) { set_last_error("out is NULL"); return GNM_E_INVAL; }
  *out = nullptr;
  if (!reg || !rec || !acc) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  // Every argument is validated and every one-time set-up (kernel attributes)
  // is done outside the capture, without running the step: a run here would
  // add into acc a second time when the step accumulates.
  int rc = classify_prepare(reg, rec, window_offsets, n_windows, p, acc, flags);
  if (rc != GNM_OK) return rc;
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_err(e, "hipStreamCreate");
  gnm_graph *g = nullptr;
  if (rc == GNM_OK) {
    g = new (std::nothrow) gnm_graph();
    if (!g) { set_last_error("host allocation failed"); rc = GNM_E_NOMEM; }
  }
  if (rc == GNM_OK) {
    e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) rc = hip_err(e, "hipStreamBeginCapture");
  }
  if (rc == GNM_OK) {
    int rc2 = flags ? gnm_classify_flag(reg, rec, window_offsets, n_windows, p, acc, threshold_bps, min_bulk_flows,
                                        flags, s)
                    : gnm_classify_aggregate(reg, rec, window_offsets, n_windows, p, acc, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc2 != GNM_OK) rc = rc2;
    else if (e != hipSuccess) rc = hip_err(e, "hipStreamEndCapture");
    g->graph = graph;
    if (rc != GNM_OK && graph) { (void)hipGraphDestroy(graph); g->graph = nullptr; }
  }
  if (rc == GNM_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_err(e, "hipGraphInstantiate");
  }
  (void)hipStreamDestroy(s);
  if (rc != GNM_OK) {
    if (g) {
      if (g->exec) (void)hipGraphExecDestroy(g->exec);
      if (g->graph) (void)hipGraphDestroy(g->graph);
      delete g;
    }
    return rc;
  }
  g->device = reg->device;
  *out = g;
  return GNM_OK;
}

extern "C" int gnm_graph_launch(gnm_graph *g, hipStream_t stream) {
  if (!g || !g->exec) { set_last_error("NULL graph"); return GNM_E_INVAL; }
  hipError_t e = hipGraphLaunch(g->exec, stream);
  if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
  return GNM_OK;
}

extern "C" int gnm_graph_free(gnm_graph *g) {
  if (!g) return GNM_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return GNM_OK;
}

extern "C" int gnm_autotune(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                            uint32_t n_windows, const gnm_params *base, gnm_acc *acc, uint32_t reps,
                            hipStream_t stream, gnm_tune_result *out) {
  if (!reg || !rec || !acc || !out) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  *out = gnm_tune_result{};
  const gnm_params b = base ? *base : gnm_params_default();
  if (reps == 0) reps = 3;
  int dev = -1, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_err(e, "device query");
  const uint32_t per_cu = reg->lds_bytes <= kLdsMax / 2 ? 2u : 1u;
  const uint32_t resident = (uint32_t)cus * per_cu;
  // candidate launch shapes: records per lane x workgroups (0 = automatic)
  const uint32_t rpts[] = {4, 2, 1};
  std::vector<uint32_t> grids = {0, resident / 2, resident * 2, resident * 4};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_err(e, "hipEventCreate");
  int rc = GNM_OK;
  uint32_t n = 0;
  float best = 1e30f;
  for (uint32_t rpt : rpts) {
    for (uint32_t grid : grids) {
      if (n >= GNM_TUNE_MAX) break;
      // with a workspace, only shapes whose partial tables fit it: every
      // candidate then merges the same way as the tuned launch will
      if (b.workspace && gnm_workspace_bytes_n(reg, rec->n, n_windows, grid) > b.workspace_bytes) continue;
      gnm_params p = b;
      p.records_per_thread = rpt;
      p.grid_blocks = grid;
      // warm-up, then the median of `reps` timed launches
      rc = gnm_classify_aggregate(reg, rec, window_offsets, n_windows, &p, acc, stream);
      if (rc != GNM_OK) break;
      std::vector<float> ms;
      for (uint32_t r = 0; r < reps && rc == GNM_OK; ++r) {
        e = hipEventRecord(e0, stream);
        if (e == hipSuccess) rc = gnm_classify_aggregate(reg, rec, window_offsets, n_windows, &p, acc, stream);
        if (e == hipSuccess && rc == GNM_OK) e = hipEventRecord(e1, stream);
        if (e == hipSuccess && rc == GNM_OK) e = hipEventSynchronize(e1);
        float t = 0;
        if (e == hipSuccess && rc == GNM_OK) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) rc = hip_err(e, "timing");
        ms.push_back(t);
      }
      if (rc != GNM_OK) break;
      std::sort(ms.begin(), ms.end());
      const float med = ms[ms.size() / 2];
      out->ms[n] = med;
      out->records_per_thread[n] = rpt;
      out->grid_blocks[n] = grid;
      if (med < best) {
        best = med;
        out->best = p;
        out->best_ms = med;
      }
      ++n;
    }
    if (rc != GNM_OK) break;
  }
  out->n_tried = n;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}
