// One whole tree in one call (Sec. 3: the levels of the first phase, then
// the leaf values and the model update of the second phase; Sec. 4: one
// split per level), and its capture into a graph the library owns.
//
// The call enqueues exactly the sequence a caller would issue level by level:
//   int16 form: the per-tree gradient codes;
//   level 0: histograms, score and argmax, the split;
//   level l >= 1: histograms (by subtraction from the previous level's when
//     asked; rows in leaf order when a partition is given), score and argmax;
//     with subtraction in the original row order the previous level's leaf
//     bit is set in the build's own row pass (cbh_apply_build_histograms_sub);
//   after every level the rows are routed by its split (the leaf bit, or the
//     move into leaf order, which writes the leaf indices at the last level);
//   the leaf solve and the approx and gradient update (for ordered boosting,
//   the update of the kept model and of the supporting approximations, and
//   the ordered gradients for the next tree).
#include <cmath>

#include "common.h"

namespace cbh {

static int fit_tree(cbh_ctx* ctx, const cbh_problem* p, cbh_part* part, int32_t precision,
                    int32_t subtract, void* const* hist, cbh_split* best, double lr, double l2,
                    double* leaf_values, int64_t* leaf_counts, uint64_t* stamps, void* stream,
                    const cbh_ordered* ord = nullptr, double* support_values = nullptr) {
    const int depth = p->depth;
    auto h = [&](int lvl) { return hist[lvl & 1]; };
    int rc = CBH_OK;
    if (precision == CBH_PREC_INT16) rc = cbh_quantize_gradients(ctx, p, stream);
    const bool fuse = part == nullptr && subtract;
    for (int lvl = 0; lvl < depth && rc == CBH_OK; ++lvl) {
        if (stamps) rc = cbh_device_timestamp(ctx, stamps + 2 * lvl, stream);
        if (rc) break;
        if (lvl == 0) {
            rc = cbh_build_histograms(ctx, p, 0, precision, h(0), stream);
        } else if (part && subtract) {
            rc = cbh_part_build_histograms_sub(ctx, part, p, lvl, precision, h(lvl - 1), h(lvl),
                                               stream);
        } else if (part) {
            rc = cbh_part_build_histograms(ctx, part, p, lvl, precision, h(lvl), stream);
        } else if (subtract) {
            rc = cbh_apply_build_histograms_sub(ctx, p, lvl, precision, h(lvl - 1),
                                                best + lvl - 1, h(lvl), stream);
        } else {
            rc = cbh_build_histograms(ctx, p, lvl, precision, h(lvl), stream);
        }
        if (!rc && stamps) rc = cbh_device_timestamp(ctx, stamps + 2 * lvl + 1, stream);
        if (!rc) rc = cbh_score_splits(ctx, p, lvl, h(lvl), precision, l2, best + lvl, nullptr,
                                       stream);
        if (rc) break;
        if (part) {
            rc = cbh_part_split(ctx, part, p, lvl, precision, best + lvl, stream);
        } else if (!fuse || lvl == depth - 1) {
            rc = cbh_apply_split(ctx, p, lvl, best + lvl, stream);
        }
    }
    if (!rc && ord)
        rc = ordered_update(ctx, ord, p, lr, l2, leaf_values, support_values,
                            (hipStream_t)stream);
    else if (!rc)
        rc = cbh_update_approx(ctx, p, h(depth - 1), precision, best + depth - 1, lr, l2,
                               leaf_values, leaf_counts, stream);
    return rc;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_fit_tree(cbh_ctx* ctx, const cbh_problem* prob, cbh_part* part, int32_t precision,
                 int32_t subtract, void* const* hist, cbh_split* best, double lr, double l2,
                 double* leaf_values, int64_t* leaf_counts, uint64_t* stamps, void* stream) {
    clear_error();
    CBH_ARG(ctx && hist && hist[0] && hist[1] && best && leaf_values, "NULL argument");
    CBH_ARG(hist[0] != hist[1], "the two histogram buffers must differ");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(std::isfinite(lr) && l2 >= 0 && std::isfinite(l2), "lr / l2 out of range");
    return fit_tree(ctx, prob, part, precision, subtract, hist, best, lr, l2, leaf_values,
                    leaf_counts, stamps, stream);
}

int cbh_fit_tree_ordered(cbh_ctx* ctx, const cbh_problem* prob, const cbh_ordered* ord,
                         cbh_part* part, int32_t precision, int32_t subtract,
                         void* const* hist, cbh_split* best, double lr, double l2,
                         double* leaf_values, double* support_values, void* stream) {
    clear_error();
    CBH_ARG(ctx && hist && hist[0] && hist[1] && best && leaf_values, "NULL argument");
    CBH_ARG(hist[0] != hist[1], "the two histogram buffers must differ");
    int rc = validate_ordered(ctx, ord, prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(std::isfinite(lr) && l2 >= 0 && std::isfinite(l2), "lr / l2 out of range");
    return fit_tree(ctx, prob, part, precision, subtract, hist, best, lr, l2, leaf_values,
                    nullptr, nullptr, stream, ord, support_values);
}

int cbh_graph_capture_tree(cbh_ctx* ctx, const cbh_problem* prob, cbh_part* part,
                           int32_t precision, int32_t subtract, void* const* hist,
                           cbh_split* best, double lr, double l2, double* leaf_values,
                           int64_t* leaf_counts, uint64_t* stamps, void* stream,
                           cbh_graph** out) {
    clear_error();
    CBH_ARG(out != nullptr, "out is NULL");
    *out = nullptr;
    CBH_ARG(stream != nullptr, "capture needs a non-default stream");
    CBH_ARG(ctx && hist && hist[0] && hist[1] && best && leaf_values, "NULL argument");
    CBH_ARG(hist[0] != hist[1], "the two histogram buffers must differ");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    rc = fit_tree(ctx, prob, part, precision, subtract, hist, best, lr, l2, leaf_values,
                  leaf_counts, stamps, stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (!rc) set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return rc ? rc : CBH_EDEVICE;
    }
    cbh_graph* g = new cbh_graph();
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    g->graph = graph;
    *out = g;
    return CBH_OK;
}

int cbh_graph_begin(cbh_ctx* ctx, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(stream != nullptr, "capture needs a non-default stream");
    CBH_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return CBH_OK;
}

int cbh_graph_end(cbh_ctx* ctx, void* stream, cbh_graph** out) {
    clear_error();
    CBH_ARG(ctx != nullptr && out != nullptr, "NULL argument");
    CBH_ARG(stream != nullptr, "capture needs a non-default stream");
    *out = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &graph);
    if (e != hipSuccess || graph == nullptr) {
        if (graph) (void)hipGraphDestroy(graph);
        set_error("hipStreamEndCapture failed: %s (a call failed under capture, or the "
                  "stream was not capturing)", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    cbh_graph* g = new cbh_graph();
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    g->graph = graph;
    *out = g;
    return CBH_OK;
}

}  // extern "C"
