// Graphs of library calls: a launch sequence captured once from a stream and
// replayed with one launch.  Only entry points that read nothing back and
// allocate nothing can be captured (their header comments say so); the
// device-driven batch sort is the one made for it.
#include <new>

#include "common.hpp"

struct ss_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int ss_graph_begin(void *stream)
{
    ss_clear_error();
    if (!stream) {
        ss_set_error("capture needs a stream other than the null stream");
        return SS_ERR_INVALID_ARG;
    }
    if (g_prof_on) {
        ss_set_error("kernel profiling is on: its events cannot be captured");
        return SS_ERR_INVALID_ARG;
    }
    SS_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return SS_OK;
}

extern "C" int ss_graph_end(void *stream, ss_graph *out)
{
    ss_clear_error();
    if (!stream || !out) {
        ss_set_error("null stream or output");
        return SS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    hipGraph_t g = nullptr;
    SS_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
    if (!g) {
        ss_set_error("capture produced no graph");
        return SS_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g);
        ss_set_error("hipGraphInstantiate: %s", hipGetErrorString(e));
        return SS_ERR_HIP;
    }
    ss_graph r = new (std::nothrow) ss_graph_s{g, x};
    if (!r) {
        hipGraphExecDestroy(x);
        hipGraphDestroy(g);
        ss_set_error("out of host memory");
        return SS_ERR_HIP;
    }
    *out = r;
    return SS_OK;
}

extern "C" int ss_graph_launch(ss_graph g, void *stream)
{
    ss_clear_error();
    if (!g) {
        ss_set_error("null graph");
        return SS_ERR_INVALID_ARG;
    }
    SS_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SS_OK;
}

extern "C" size_t ss_graph_nodes(ss_graph g)
{
    size_t cnt = 0;
    if (g && hipGraphGetNodes(g->graph, nullptr, &cnt) != hipSuccess) cnt = 0;
    return cnt;
}

extern "C" void ss_graph_destroy(ss_graph g)
{
    if (!g) return;
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
}
