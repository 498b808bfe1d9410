// Many independent join instances at once (batched serving), and the plan
// autotuner.
//
// A batch owns a few streams of default priority.  Its plans are assigned to
// the streams longest-first by an estimate of their work (the register-tile
// QR dominates: items x columns^2 summed over the head/tail tasks, plus the
// stack of the post-processing TSQR), so the small kernels of many
// instances run side by side.  A batch pass forks from the caller's stream
// with an event, runs every plan's pass on its stream and joins back with
// one event per stream; the same sequence can be captured once into a HIP
// graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

namespace figaro {
figaro_status set_error(figaro_plan_s *p, figaro_status st, const std::string &msg);
extern thread_local std::string g_thread_error;
}  // namespace figaro

using namespace figaro;

struct figaro_batch_s {
    std::vector<figaro_plan_t> plans;
    std::vector<double> cost;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_of;       // per plan
    std::vector<int> order;           // plans, largest estimated work first
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

namespace {

figaro_status batch_error(figaro_status st, const std::string &msg) {
    g_thread_error = msg;
    return st;
}

double plan_cost(const figaro_plan_s *p) {
    double c = 0.0;
    for (const RelPlan &R : p->rel)
        for (const Task *T : {&R.a2, &R.a4})
            if (T->active && !T->levels.empty())
                c += (double)T->levels[0].items * T->ncols * T->ncols;
    c += (double)p->stack_rows * p->n * p->n;
    return c + 1.0;
}

// Per-launch timing records events on the launch stream into a plan's pool
// and reads them back on the host; a batch spreads its plans over several
// streams, so batches refuse plans with timing enabled (eager passes and
// capture alike).
bool any_profiling(const figaro_batch_s *b) {
    for (const figaro_plan_s *p : b->plans)
        if (!p->prof_start.empty()) return true;
    return false;
}

void release_graph(figaro_batch_s *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// One pass over every plan of the batch, forked from and joined back to `s`.
template <class F>
figaro_status batch_pass(figaro_batch_s *b, hipStream_t s, F &&one) {
    if (hipEventRecord(b->fork, s) != hipSuccess) return batch_error(FIGARO_EHIP, "event record failed");
    for (hipStream_t t : b->streams)
        if (hipStreamWaitEvent(t, b->fork, 0) != hipSuccess) return batch_error(FIGARO_EHIP, "stream wait failed");
    figaro_status first_error = FIGARO_OK;
    std::string msg;
    for (int i : b->order) {
        figaro_status st = one(i, b->streams[b->stream_of[i]]);
        if (st != FIGARO_OK && first_error == FIGARO_OK) {
            first_error = st;
            const char *e = figaro_last_error(b->plans[i]);
            msg = "instance " + std::to_string(i) + ": " + (e ? e : "");
        }
    }
    // join every stream back, also after an error, so no stream is left
    // forked (and a capture can end)
    for (size_t k = 0; k < b->streams.size(); ++k) {
        if (hipEventRecord(b->join[k], b->streams[k]) != hipSuccess ||
            hipStreamWaitEvent(s, b->join[k], 0) != hipSuccess)
            return batch_error(FIGARO_EHIP, "stream join failed");
    }
    return first_error == FIGARO_OK ? FIGARO_OK : batch_error(first_error, msg);
}

}  // namespace

extern "C" {

figaro_status figaro_batch_create(figaro_batch_t *out, int32_t count, const figaro_plan_t *plans, int32_t streams) {
    if (!out) return batch_error(FIGARO_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !plans) return batch_error(FIGARO_EINVAL, "need at least one plan");
    std::vector<figaro_plan_t> v(plans, plans + count);
    for (int i = 0; i < count; ++i) {
        if (!v[i]) return batch_error(FIGARO_EINVAL, "plan " + std::to_string(i) + " is NULL");
        if (v[i]->analyze_only) return batch_error(FIGARO_EINVAL, "plan " + std::to_string(i) + " is analyze-only");
    }
    {
        std::vector<figaro_plan_t> s = v;
        std::sort(s.begin(), s.end());
        if (std::adjacent_find(s.begin(), s.end()) != s.end())
            return batch_error(FIGARO_EINVAL, "a plan appears twice (plans own their workspace)");
    }
    const int ns = std::max(1, std::min<int>(streams > 0 ? streams : 8, count));
    figaro_batch_s *b = new figaro_batch_s();
    b->plans = v;
    (void)hipGetDevice(&b->device);
    for (int k = 0; k < ns; ++k) {
        hipStream_t t;
        if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) {
            figaro_batch_destroy(b);
            return batch_error(FIGARO_EHIP, "stream creation failed");
        }
        b->streams.push_back(t);
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            figaro_batch_destroy(b);
            return batch_error(FIGARO_EHIP, "event creation failed");
        }
        b->join.push_back(e);
    }
    if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
        figaro_batch_destroy(b);
        return batch_error(FIGARO_EHIP, "event creation failed");
    }
    // longest processing time first onto the least loaded stream
    b->cost.resize(count);
    for (int i = 0; i < count; ++i) b->cost[i] = plan_cost(v[i]);
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
    std::vector<double> load(ns, 0.0);
    b->stream_of.assign(count, 0);
    for (int i : b->order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->stream_of[i] = k;
        load[k] += b->cost[i];
    }
    *out = b;
    return FIGARO_OK;
}

void figaro_batch_destroy(figaro_batch_t b) {
    if (!b) return;
    release_graph(b);
    for (hipStream_t t : b->streams) (void)hipStreamDestroy(t);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

int32_t figaro_batch_stream_of(figaro_batch_t b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->plans.size()) return -1;
    return b->stream_of[i];
}

figaro_status figaro_r_batched(figaro_batch_t b, const double *const *const *values, const int64_t *const *ld,
                               double *const *R, hipStream_t stream) {
    if (!b || !values || !ld || !R) return batch_error(FIGARO_EINVAL, "NULL argument");
    if (any_profiling(b)) return batch_error(FIGARO_EINVAL, "disable profiling on the batch's plans");
    return batch_pass(b, stream, [&](int i, hipStream_t t) {
        if (!values[i] || !ld[i] || !R[i]) return set_error(b->plans[i], FIGARO_EINVAL, "NULL argument");
        return run_forward(b->plans[i], values[i], ld[i], R[i], t);
    });
}

figaro_status figaro_r_backward_batched(figaro_batch_t b, const double *const *const *values,
                                        const int64_t *const *ld, const double *const *R, const double *const *dR,
                                        double *const *const *dvalues, const int64_t *const *ld_dvalues,
                                        hipStream_t stream) {
    if (!b || !values || !ld || !R || !dR || !dvalues || !ld_dvalues)
        return batch_error(FIGARO_EINVAL, "NULL argument");
    if (any_profiling(b)) return batch_error(FIGARO_EINVAL, "disable profiling on the batch's plans");
    return batch_pass(b, stream, [&](int i, hipStream_t t) {
        if (!values[i] || !ld[i] || !R[i] || !dR[i] || !dvalues[i] || !ld_dvalues[i])
            return set_error(b->plans[i], FIGARO_EINVAL, "NULL argument");
        return run_backward(b->plans[i], values[i], ld[i], R[i], dR[i], dvalues[i], ld_dvalues[i], t);
    });
}

figaro_status figaro_batch_capture(figaro_batch_t b, const double *const *const *values, const int64_t *const *ld,
                                   double *const *R, hipStream_t stream) {
    if (!b || !values || !ld || !R) return batch_error(FIGARO_EINVAL, "NULL argument");
    if (!stream) return batch_error(FIGARO_EINVAL, "capture needs a stream other than the null stream");
    for (figaro_plan_t p : b->plans)
        if (!p->prof_start.empty()) return batch_error(FIGARO_EINVAL, "disable profiling before capturing");
    release_graph(b);
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return batch_error(FIGARO_EHIP, "stream capture could not begin");
    figaro_status st = figaro_r_batched(b, values, ld, R, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &g);
    if (st != FIGARO_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g) return batch_error(FIGARO_EHIP, "stream capture failed");
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        release_graph(b);
        return batch_error(FIGARO_EHIP, "graph instantiation failed");
    }
    return FIGARO_OK;
}

figaro_status figaro_batch_launch(figaro_batch_t b, hipStream_t stream) {
    if (!b || !b->exec) return batch_error(FIGARO_EINVAL, "no captured graph");
    return hipGraphLaunch(b->exec, stream) == hipSuccess ? FIGARO_OK
                                                         : batch_error(FIGARO_EHIP, "graph launch failed");
}

// ---------------------------------------------------------------------------
// Autotuner: build the plan under several option sets, time the forward pass
// of each on the caller's values, keep the fastest.
// ---------------------------------------------------------------------------
figaro_status figaro_plan_create_tuned(figaro_plan_t *out, int32_t r, const figaro_relation_desc *rels,
                                       const double *const *values, const int64_t *ld, int32_t ncandidates,
                                       const figaro_plan_options *candidates, int32_t reps, hipStream_t stream) {
    if (!out) return batch_error(FIGARO_EINVAL, "out is NULL");
    *out = nullptr;
    if (r < 1 || !rels || !values || !ld) return batch_error(FIGARO_EINVAL, "NULL argument");
    std::vector<figaro_plan_options> cand;
    if (ncandidates > 0 && candidates) {
        cand.assign(candidates, candidates + ncandidates);
    } else {
        for (int variant : {0, 2})
            for (int cap : {512, 1024, 2048}) {
                figaro_plan_options o{};
                o.variant = variant;
                o.waves_per_task = cap;
                cand.push_back(o);
            }
    }
    for (auto &o : cand) o.analyze_only = 0;
    reps = std::max(1, reps);
    figaro_plan_t best = nullptr;
    double best_ms = 0.0;
    figaro_plan_options best_opt{};
    std::vector<double *> buf(r, nullptr);
    std::vector<int64_t> bld(r, 1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    figaro_status result = FIGARO_OK;
    std::string msg;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        result = FIGARO_EHIP;
        msg = "event creation failed";
    }
    double *Rtmp = nullptr;
    for (size_t ci = 0; ci < cand.size() && result == FIGARO_OK; ++ci) {
        figaro_plan_t p = nullptr;
        figaro_status st = figaro_plan_create(&p, r, rels, &cand[ci], stream);
        if (st != FIGARO_OK) {
            // an option set this instance cannot use; the first error is kept
            // in case no candidate works
            if (msg.empty()) msg = g_thread_error;
            continue;
        }
        if (!Rtmp) {
            // plan-order copies of the values (the sort order depends on the
            // keys only, so it is the same for every candidate)
            const int n = figaro_plan_num_cols(p);
            if (hipMalloc((void **)&Rtmp, sizeof(double) * (size_t)n * n) != hipSuccess) {
                figaro_plan_destroy(p);
                result = FIGARO_ENOMEM;
                msg = "hipMalloc";
                break;
            }
            for (int i = 0; i < r && result == FIGARO_OK; ++i) {
                const int64_t m = std::max<int64_t>(figaro_plan_rows(p, i), 1);
                bld[i] = m;
                if (hipMalloc((void **)&buf[i], sizeof(double) * (size_t)m * rels[i].num_cols) != hipSuccess) {
                    result = FIGARO_ENOMEM;
                    msg = "hipMalloc";
                } else if (figaro_permute_values(p, i, values[i], ld[i], buf[i], bld[i], stream) != FIGARO_OK) {
                    result = FIGARO_EHIP;
                    msg = "permutation failed";
                }
            }
            if (result != FIGARO_OK) {
                figaro_plan_destroy(p);
                break;
            }
        }
        const double *const *pv = buf.data();
        st = figaro_r(p, pv, bld.data(), Rtmp, stream);   // warm-up
        float ms = 0.0f;
        if (st == FIGARO_OK && hipEventRecord(e0, stream) == hipSuccess) {
            for (int k = 0; k < reps && st == FIGARO_OK; ++k) st = figaro_r(p, pv, bld.data(), Rtmp, stream);
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                st = FIGARO_EHIP;
        }
        if (st != FIGARO_OK) {
            figaro_plan_destroy(p);
            result = st;
            msg = "timing a candidate failed";
            break;
        }
        const double t = (double)ms / reps;
        if (!best || t < best_ms) {
            if (best) figaro_plan_destroy(best);
            best = p;
            best_ms = t;
            best_opt = cand[ci];
        } else {
            figaro_plan_destroy(p);
        }
    }
    (void)hipStreamSynchronize(stream);
    for (double *q : buf) if (q) (void)hipFree(q);
    if (Rtmp) (void)hipFree(Rtmp);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (result != FIGARO_OK) {
        if (best) figaro_plan_destroy(best);
        return batch_error(result, msg);
    }
    if (!best) return batch_error(FIGARO_EUNSUPPORTED, "no candidate option set works: " + msg);
    best->tuned_ms = best_ms;
    best->tuned_options = best_opt;
    *out = best;
    return FIGARO_OK;
}

figaro_status figaro_plan_tuning(figaro_plan_t p, figaro_plan_options *chosen, double *ms) {
    if (!p || !chosen || !ms) return set_error(p, FIGARO_EINVAL, "bad argument");
    if (p->tuned_ms < 0.0) return set_error(p, FIGARO_EINVAL, "the plan was not built by the autotuner");
    *chosen = p->tuned_options;
    *ms = p->tuned_ms;
    return FIGARO_OK;
}

}  // extern "C"
