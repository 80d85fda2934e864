// LM iterations captured in a HIP graph.  poba_lm_step makes no host
// synchronisation and no memory set or copy, so a run of steps can be
// recorded once by stream capture and replayed with one launch: the launch
// cost of the ~40 kernels per step (per batch of problems) is paid once.
#include "common.hpp"

struct poba_lm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

poba_status poba_lm_graph_create(poba_problem p, double* cams, double* lms, poba_lm_state* st,
                                 const poba_lm_options* o, int32_t n_steps, poba_lm_graph* out) {
    (void)hipGetLastError();  // report only this call's errors
    if (!p || !cams || !lms || !st || !o || !out || n_steps < 1 || n_steps > 1000) return POBA_ERR_INVALID_ARG;
    *out = nullptr;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return POBA_ERR_HIP;
    const bool profiling = p->profiling;
    p->profiling = false;  // events are not recorded into the graph
    poba_status rc = POBA_OK;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = POBA_ERR_HIP;
    } else {
        for (int32_t k = 0; k < n_steps && rc == POBA_OK; ++k)
            rc = poba_lm_step(p, cams, lms, st, o, reinterpret_cast<poba_stream>(cs));
        if (hipStreamEndCapture(cs, &graph) != hipSuccess && rc == POBA_OK) rc = POBA_ERR_HIP;
    }
    p->profiling = profiling;
    hipGraphExec_t exec = nullptr;
    if (rc == POBA_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = POBA_ERR_HIP;
    (void)hipStreamDestroy(cs);
    if (rc != POBA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    auto* g = new poba_lm_graph_s();
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return POBA_OK;
}

poba_status poba_lm_graph_launch(poba_lm_graph g, poba_stream stream) {
    if (!g) return POBA_ERR_INVALID_ARG;
    return hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? POBA_OK : POBA_ERR_HIP;
}

poba_status poba_lm_graph_destroy(poba_lm_graph g) {
    if (!g) return POBA_ERR_INVALID_ARG;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return POBA_OK;
}

}  // extern "C"
