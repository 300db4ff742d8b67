// Histogram launch autotuner.
//
// It walks one tree of a problem level by level. At every level it times the
// histogram build (main launch plus the partial merge) in the mode the tree
// uses (direct, or by subtraction from the previous level) for each distinct
// launch plan reachable from a grid of knobs — LDS bytes per block, the
// number of blocks aimed at, the least rows per block, the cap on partial-tile
// volume and the LDS replicas per cell — keeps the fastest, then builds that
// level with it, scores it and applies the split so the next level sees real
// leaves. Results are keyed by (F, B, K, level, precision, floor(log2 n),
// mode) and can be saved to and loaded from a small JSON file.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

static bool parse_field(const std::string& obj, const char* key, long long* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    const size_t c = obj.find(':', p + k.size());
    if (c == std::string::npos) return false;
    return sscanf(obj.c_str() + c + 1, " %lld", out) == 1;
}

static int save_table(const cbh_ctx* ctx, const char* path) {
    FILE* f = fopen(path, "w");
    CBH_REQUIRE(f != nullptr, CBH_EINVAL, "cannot write %s", path);
    fprintf(f, "[\n");
    size_t i = 0;
    for (const auto& kv : ctx->tuned) {
        const TuneKey& k = kv.first;
        const HistKnobs& v = kv.second;
        fprintf(f,
                "  {\"F\": %d, \"B\": %d, \"K\": %d, \"level\": %d, \"precision\": %d, "
                "\"sub\": %d, "
                "\"log2n\": %d, \"lds_budget\": %d, \"max_fb\": %d, \"target_blocks\": %d, "
                "\"min_rows\": %lld, \"partial_pct\": %d, \"max_rep\": %d, "
                "\"rep_target\": %d, \"kernel\": %d, \"lpf_w\": %d%s}%s\n",
                std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                std::get<6>(k), std::get<5>(k), v.lds_budget, v.max_fb, v.target_blocks, (long long)v.min_rows,
                v.partial_pct, v.max_rep, v.rep_target, v.kernel, v.lpf_w,
                ctx->tuned_note.count(k) ? ctx->tuned_note.at(k).c_str() : "",
                ++i < ctx->tuned.size() ? "," : "");
    }
    fprintf(f, "]\n");
    fclose(f);
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_set_hist_knobs(cbh_ctx* ctx, int32_t lds_budget, int32_t target_blocks,
                       int64_t min_rows, int32_t partial_pct, int32_t max_rep,
                       int32_t rep_target, int32_t kernel, int32_t lpf_w) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    if (lds_budget == 0) {
        ctx->force_knobs = false;
        return CBH_OK;
    }
    CBH_ARG(lds_budget > 0 && target_blocks > 0 && min_rows > 0 && partial_pct > 0 &&
                max_rep > 0 && rep_target > 0 && (max_rep & (max_rep - 1)) == 0,
            "knobs must be > 0 and max_rep a power of two");
    CBH_ARG(kernel == 0 || kernel == 1, "kernel must be 0 or 1");
    CBH_ARG(lpf_w == 0 || lpf_w == 4 || lpf_w == 8 || lpf_w == 16 || lpf_w == 32,
            "lpf_w must be 0, 4, 8, 16 or 32");
    HistKnobs kn;
    kn.lds_budget = lds_budget;
    kn.target_blocks = target_blocks;
    kn.min_rows = min_rows;
    kn.partial_pct = partial_pct;
    kn.max_rep = max_rep;
    kn.rep_target = rep_target;
    kn.kernel = kernel;
    kn.lpf_w = lpf_w;
    ctx->forced = kn;
    ctx->force_knobs = true;
    return CBH_OK;
}

int cbh_autotune_load(cbh_ctx* ctx, const char* cache_path) {
    clear_error();
    CBH_ARG(ctx && cache_path, "NULL argument");
    FILE* f = fopen(cache_path, "r");
    CBH_ARG(f != nullptr, "cannot open %s", cache_path);
    std::string text;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, r);
    fclose(f);
    size_t pos = 0;
    int loaded = 0;
    while ((pos = text.find('{', pos)) != std::string::npos) {
        const size_t end = text.find('}', pos);
        CBH_ARG(end != std::string::npos, "malformed autotune file");
        const std::string obj = text.substr(pos, end - pos + 1);
        long long F, B, K, lvl, prec, l2n, lds, fb, tb, mr, pp, mrep = 32, rtg = 32, sub = 0;
        long long kern = 1, lw = 0;
        CBH_ARG(parse_field(obj, "F", &F) && parse_field(obj, "B", &B) &&
                    parse_field(obj, "K", &K) && parse_field(obj, "level", &lvl) &&
                    parse_field(obj, "precision", &prec) && parse_field(obj, "log2n", &l2n) &&
                    parse_field(obj, "lds_budget", &lds) && parse_field(obj, "max_fb", &fb) &&
                    parse_field(obj, "target_blocks", &tb) && parse_field(obj, "min_rows", &mr) &&
                    parse_field(obj, "partial_pct", &pp),
                "malformed autotune entry");
        parse_field(obj, "max_rep", &mrep);      // optional
        parse_field(obj, "rep_target", &rtg);    // optional
        parse_field(obj, "sub", &sub);           // optional
        parse_field(obj, "kernel", &kern);       // optional
        parse_field(obj, "lpf_w", &lw);          // optional
        CBH_ARG(lds > 0 && fb > 0 && tb > 0 && mr > 0 && pp > 0 && mrep > 0,
                "bad autotune values");
        HistKnobs kn;
        kn.lds_budget = (int32_t)lds;
        kn.max_fb = (int32_t)fb;
        kn.target_blocks = (int32_t)tb;
        kn.min_rows = mr;
        kn.partial_pct = (int32_t)pp;
        kn.max_rep = (int32_t)mrep;
        kn.rep_target = (int32_t)std::max<long long>(1, rtg);
        kn.kernel = kern != 0 ? 1 : 0;
        kn.lpf_w = (int32_t)std::max<long long>(0, std::min<long long>(32, lw));
        ctx->tuned[TuneKey{(int32_t)F, (int32_t)B, (int32_t)K, (int32_t)lvl, (int32_t)prec,
                           (int32_t)l2n, (int32_t)(sub != 0)}] = kn;
        ++loaded;
        pos = end + 1;
    }
    return CBH_OK;
}

int cbh_autotune(cbh_ctx* ctx, const cbh_problem* prob, int32_t precision, int32_t subtract,
                 const char* cache_path, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    CBH_REQUIRE(!packed_bins(prob), CBH_EUNSUPPORTED,
                "autotuning takes byte bins (packed bins have one kernel and its default plan)");
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int F = prob->n_features, B = prob->max_bins, K = prob->K;
    const int rmse = count_stat(prob);
    std::vector<int32_t> budgets;
    for (int32_t v : {32 * 1024, 64 * 1024, 96 * 1024, 128 * 1024, 160 * 1024})
        if (v <= ctx->max_lds) budgets.push_back(v);
    const int32_t targets[] = {256, 512, 1024};
    const int64_t min_rows[] = {16384, 32768, 65536};
    const int32_t pcts[] = {12, 25, 50};
    const int32_t reps[] = {1, 8, 32};
    const int32_t lpf_ws[] = {32, 16, 8, 4};
    CBH_REQUIRE(tile_lds_bytes(precision, rmse, K, B, 1) <= ctx->max_lds, CBH_EUNSUPPORTED,
                "leaf row does not fit in LDS");
    const int64_t hist_bytes =
        hist_elems(1 << (prob->depth - 1), F, B, K) * hist_elem_bytes(precision);
    // two level histograms (current, parent), the split of every level, parent sides
    void* hbuf[2] = {nullptr, nullptr};
    cbh_split* splits = nullptr;
    uint8_t* side = nullptr;
    const int64_t max_half = int64_t(1) << std::max(0, prob->depth - 2);
    CBH_HIP(hipMalloc(&hbuf[0], (size_t)std::max<int64_t>(hist_bytes, 256)));
    CBH_HIP(hipMalloc(&hbuf[1], (size_t)std::max<int64_t>(hist_bytes, 256)));
    CBH_HIP(hipMalloc((void**)&splits, sizeof(cbh_split) * prob->depth));
    CBH_HIP(hipMalloc((void**)&side, (size_t)std::max<int64_t>(max_half, 256)));
    uint16_t* codes = nullptr;      // row codes of the lanes-over-features kernel
    CBH_HIP(hipMalloc((void**)&codes, (size_t)prob->n * 2));
    hipEvent_t e0, e1;
    CBH_HIP(hipEventCreate(&e0));
    CBH_HIP(hipEventCreate(&e1));
    int32_t nb = 0;
    while ((int64_t(1) << (nb + 1)) <= prob->n) ++nb;
    for (int level = 0; level < prob->depth && rc == CBH_OK; ++level) {
        const int sub = (subtract && level > 0) ? 1 : 0;
        const int L = sub ? 1 << (level - 1) : 1 << level;
        void* out = hbuf[level & 1];
        const void* parent = sub ? hbuf[(level - 1) & 1] : nullptr;
        float best_ms = 1e30f;
        HistKnobs best_kn = ctx->knobs;
        // candidate knob sets: the rows-over-lanes kernel over LDS budget x
        // replicas, and the features-over-lanes kernel over lane-group width;
        // both over blocks aimed at x rows per block x partial volume
        std::vector<HistKnobs> cands;
        for (int32_t tb : targets)
            for (int64_t mr : min_rows)
                for (int32_t pp : pcts) {
                    HistKnobs kn = ctx->knobs;
                    kn.target_blocks = tb;
                    kn.min_rows = mr;
                    kn.partial_pct = pp;
                    kn.kernel = 0;
                    for (size_t ib = 0; ib < budgets.size(); ++ib)
                        for (int32_t mrp : reps) {
                            kn.lds_budget = budgets[ib];
                            kn.max_rep = mrp;
                            kn.rep_target = mrp;
                            cands.push_back(kn);
                        }
                    kn.kernel = 1;
                    kn.max_rep = kn.rep_target = 1;
                    kn.lds_budget = ctx->max_lds;
                    for (int32_t w : lpf_ws) {
                        kn.lpf_w = w;
                        cands.push_back(kn);
                    }
                }
        std::set<std::tuple<int, int, int, int64_t, int>> seen;
        for (size_t ci = 0; ci < cands.size() && rc == CBH_OK; ++ci) {
            const HistKnobs kn = cands[ci];
            const HistPlan plan = plan_hist(kn, prob->n, F, B, K, L, precision, rmse,
                                            ctx->max_lds);
            if (!seen.insert({plan.kind, plan.fb, plan.lt, plan.rows_per_chunk, plan.rep})
                     .second)
                continue;
            const int64_t part = int64_t(plan.n_chunks) * L * F * B *
                                 plan.words_per_cell * 4;
            if (part > ctx->ws_limit / 2) continue;
            rc = ensure_ws(ctx, part, s);
            if (rc) break;
            // warm-up, then the mean of 3 timed runs
            rc = launch_hist(ctx, prob, level, precision, plan, out, ctx->ws, s, parent,
                             sub ? side : nullptr, codes, sub ? splits + level - 1 : nullptr);
            if (rc) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 3 && !rc; ++r)
                rc = launch_hist(ctx, prob, level, precision, plan, out, ctx->ws, s,
                                 parent, sub ? side : nullptr, codes,
                                 sub ? splits + level - 1 : nullptr);
            (void)hipEventRecord(e1, s);
            if (rc) break;
            if (hipEventSynchronize(e1) != hipSuccess) {
                set_error("autotune timing failed");
                rc = CBH_EDEVICE;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best_kn = kn;
            }
        }
        if (rc) break;
        ctx->tuned[TuneKey{F, B, K, level, precision, nb, sub}] = best_kn;
        // build this level with the chosen plan, score it and apply its split
        const HistPlan plan = plan_hist(best_kn, prob->n, F, B, K, L, precision, rmse,
                                        ctx->max_lds);
        {
            char note[256];
            snprintf(note, sizeof(note),
                     ", \"plan_kind\": %d, \"plan_fb\": %d, \"plan_lt\": %d, \"plan_chunks\": %d, "
                     "\"plan_rows\": %lld, \"plan_rep\": %d, \"plan_blocks\": %lld, "
                     "\"plan_lds\": %lld, \"us\": %.1f",
                     plan.kind, plan.fb, plan.lt, plan.n_chunks, (long long)plan.rows_per_chunk, plan.rep,
                     (long long)plan.n_blocks, (long long)plan.lds_bytes, best_ms * 1000.f / 3.f);
            ctx->tuned_note[TuneKey{F, B, K, level, precision, nb, sub}] = note;
        }
        rc = ensure_ws(ctx, int64_t(plan.n_chunks) * L * F * B * plan.words_per_cell * 4 +
                                score_scratch_bytes(prob) + 256, s);
        if (!rc) rc = launch_hist(ctx, prob, level, precision, plan, out, ctx->ws, s, parent,
                                  sub ? side : nullptr, codes,
                                  sub ? splits + level - 1 : nullptr);
        if (!rc) rc = launch_score(ctx, prob, level, out, precision, 1.0, splits + level, nullptr,
                                   ctx->ws, s);
        if (!rc) rc = launch_apply(ctx, prob, level, splits + level, s);
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(hbuf[0]);
    (void)hipFree(hbuf[1]);
    (void)hipFree(splits);
    (void)hipFree(side);
    (void)hipFree(codes);
    if (rc) return rc;
    if (cache_path) return save_table(ctx, cache_path);
    return CBH_OK;
}

}  // extern "C"
