// Several independent cells in one launch sequence: the applies of all cells
// are captured into one hipGraph, each cell's kernels on a stream of its own
// forked from the batch stream, so that small cells run side by side and fill
// the GPU.  The graph is replayed while the arguments, the set of active
// cells and every cell's workspaces stay the same; bse_batch_davidson drives
// all cells' Davidson iterations in lockstep through it.
#include <algorithm>

#include "ctx.hpp"

namespace bse {

static void batch_drop_graph(bse_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->g_prec = -1;
}

void batch_create(bse_batch *b, bse_ctx *const *ctxs, int n, hipStream_t stream) {
    BSE_REQUIRE(n >= 1 && n <= 256, BSE_ERR_ARG, "a batch holds 1 to 256 contexts");
    BSE_REQUIRE(stream != nullptr, BSE_ERR_ARG, "a batch needs a non-default stream");
    b->stream = stream;
    for (int i = 0; i < n; ++i) {
        BSE_REQUIRE(ctxs[i] != nullptr, BSE_ERR_ARG, "null context %d in the batch", i);
        for (int j = 0; j < i; ++j)
            BSE_REQUIRE(ctxs[j] != ctxs[i], BSE_ERR_ARG, "context %d appears twice", i);
        BSE_REQUIRE(ctxs[i]->device == ctxs[0]->device, BSE_ERR_ARG,
                    "all contexts of a batch must be on one device");
        b->cells.push_back(ctxs[i]);
    }
    BSE_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    b->side.resize(n, nullptr);
    b->join.resize(n, nullptr);
    for (int i = 0; i < n; ++i) {
        // default priority, like every other stream of the library
        BSE_HIP(hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking));
        BSE_HIP(hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming));
    }
}

void batch_free(bse_batch *b) {
    batch_drop_graph(b);
    for (auto s : b->side)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : b->join)
        if (e) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    b->side.clear();
    b->join.clear();
    b->fork = nullptr;
}

static int ws_gen(const bse_ctx *c) { return c->ws64.gen + c->ws32.gen + c->aws.gen; }

// Apply cell i's operator to n_vec[i] vectors, in[i] -> out[i], for every i
// with active[i] (all when active is null).  Returns after completion.
void batch_apply(bse_batch *b, const int *n_vec, const void *const *in, void *const *out,
                 int prec, const char *active) {
    const int nc = (int)b->cells.size();
    BSE_REQUIRE(prec == BSE_FP64 || prec == BSE_FP32 || prec == BSE_BF16X3, BSE_ERR_ARG,
                "unknown precision %d", prec);
    std::vector<char> act(nc, 1);
    if (active)
        for (int i = 0; i < nc; ++i) act[i] = active[i] ? 1 : 0;
    for (int i = 0; i < nc; ++i) {
        if (!act[i]) continue;
        bse_ctx *c = b->cells[i];
        BSE_REQUIRE(n_vec[i] >= 1, BSE_ERR_ARG, "cell %d: n_vec must be >= 1", i);
        BSE_REQUIRE(in[i] && out[i] && in[i] != out[i], BSE_ERR_ARG,
                    "cell %d: A_in/A_out must be distinct device buffers", i);
        BSE_REQUIRE(prec == BSE_FP64 ? c->have_tau64 : c->have_tau32, BSE_ERR_STATE,
                    "cell %d: apply needs bse_screen_pairs in the requested precision", i);
    }
    if (!b->use_graph) {
        for (int i = 0; i < nc; ++i)
            if (act[i]) ctx_apply(b->cells[i], n_vec[i], in[i], out[i], prec);
        for (int i = 0; i < nc; ++i)
            if (act[i]) BSE_HIP(hipStreamSynchronize(b->cells[i]->stream));
        return;
    }
    bool hit = b->gexec != nullptr && b->g_prec == prec && (int)b->g_active.size() == nc;
    for (int i = 0; hit && i < nc; ++i) {
        hit = b->g_active[i] == act[i];
        if (hit && act[i])
            hit = b->g_nvec[i] == n_vec[i] && b->g_in[i] == in[i] && b->g_out[i] == out[i] &&
                  b->g_gen[i] == ws_gen(b->cells[i]);
    }
    if (!hit) {
        // eager runs size every workspace; then capture the same launches
        for (int i = 0; i < nc; ++i)
            if (act[i]) ctx_apply(b->cells[i], n_vec[i], in[i], out[i], prec);
        for (int i = 0; i < nc; ++i)
            if (act[i]) BSE_HIP(hipStreamSynchronize(b->cells[i]->stream));
        batch_drop_graph(b);
        std::vector<int> gen(nc, 0);
        for (int i = 0; i < nc; ++i) gen[i] = ws_gen(b->cells[i]);
        std::vector<hipStream_t> saved(nc);
        for (int i = 0; i < nc; ++i) saved[i] = b->cells[i]->stream;
        BSE_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        try {
            BSE_HIP(hipEventRecord(b->fork, b->stream));
            for (int i = 0; i < nc; ++i) {
                if (!act[i]) continue;
                BSE_HIP(hipStreamWaitEvent(b->side[i], b->fork, 0));
                b->cells[i]->stream = b->side[i];
                ctx_apply(b->cells[i], n_vec[i], in[i], out[i], prec);
                b->cells[i]->stream = saved[i];
                BSE_HIP(hipEventRecord(b->join[i], b->side[i]));
                BSE_HIP(hipStreamWaitEvent(b->stream, b->join[i], 0));
            }
        } catch (...) {
            for (int i = 0; i < nc; ++i) b->cells[i]->stream = saved[i];
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(b->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        BSE_HIP(hipStreamEndCapture(b->stream, &b->graph));
        BSE_HIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        for (int i = 0; i < nc; ++i)
            BSE_REQUIRE(!act[i] || ws_gen(b->cells[i]) == gen[i], BSE_ERR_HIP,
                        "cell %d: apply workspaces changed during capture", i);
        b->g_prec = prec;
        b->g_active = act;
        b->g_nvec.assign(n_vec, n_vec + nc);
        b->g_in.assign(in, in + nc);
        b->g_out.assign(out, out + nc);
        b->g_gen = gen;
    }
    BSE_HIP(hipGraphLaunch(b->gexec, b->stream));
    BSE_HIP(hipStreamSynchronize(b->stream));
}

void batch_set_graph(bse_batch *b, bool on) {
    if (!on) batch_drop_graph(b);
    b->use_graph = on;
}

}  // namespace bse
