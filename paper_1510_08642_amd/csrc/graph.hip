// Capture and replay of library call sequences as HIP graphs.
#include "common.hpp"
#include "ddqd.h"

struct ddqd_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace ddqd {
int check_device();
void clear_error();
}  // namespace ddqd

using namespace ddqd;

extern "C" {

int ddqd_graph_begin(void* stream) {
  clear_error();
  if (!stream) return set_error(DDQD_E_ARG, "graph capture needs a non-null stream");
  int rc = check_device();
  if (rc) return rc;
  const hipError_t e =
      hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess)
    return set_error(DDQD_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  return DDQD_OK;
}

int ddqd_graph_end(void* stream, ddqd_graph_t* graph) {
  clear_error();
  if (!graph) return set_error(DDQD_E_ARG, "graph: null output pointer");
  *graph = nullptr;
  if (!stream) return set_error(DDQD_E_ARG, "graph capture needs a non-null stream");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
  if (e != hipSuccess || !g)
    return set_error(DDQD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(DDQD_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *graph = new ddqd_graph{g, x};
  return DDQD_OK;
}

int ddqd_graph_launch(ddqd_graph_t graph, void* stream) {
  clear_error();
  if (!graph) return set_error(DDQD_E_ARG, "graph: null handle");
  const hipError_t e = hipGraphLaunch(graph->exec, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(DDQD_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return DDQD_OK;
}

int ddqd_graph_destroy(ddqd_graph_t graph) {
  clear_error();
  if (!graph) return DDQD_OK;
  (void)hipGraphExecDestroy(graph->exec);
  (void)hipGraphDestroy(graph->graph);
  delete graph;
  return DDQD_OK;
}

}  // extern "C"
