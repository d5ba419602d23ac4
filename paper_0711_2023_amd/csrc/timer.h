// HIP events around the kernels and phases of a decomposition's sweeps, on
// the call's stream (opts.timing, opts.trace of tucker.h). Shared by the
// drivers of every order.
#pragma once

#include "../../include/tucker.h"
#include "common.h"

#include <vector>

namespace tk {

// HIP events around the phases of a sweep, on the call's stream. Each pair
// carries its phase, the mode it serves and its element type; collect()
// (after a stream synchronisation, once per sweep) sums them per phase and
// appends them to the caller's trace when one is given.
enum TimedKind { kProj = TK_PHASE_PROJECT, kTtmc = TK_PHASE_TTMC2, kGram = TK_PHASE_GRAM, kEig = TK_PHASE_EIG,
                 kCore = TK_PHASE_CORE };
struct Timer {
    bool on;
    hipStream_t s;
    tk_trace *tr;
    std::vector<hipEvent_t> ev;
    struct Tag {
        int kind, mode, prec;
    };
    std::vector<Tag> tag;
    size_t used = 0;
    double ms[5] = {0, 0, 0, 0, 0};
    int64_t calls[5] = {0, 0, 0, 0, 0};
    double sweep_ttmc[64] = {};  // TTMc time (projections + second stage) per collect() = per sweep
    int sweeps = 0;
    Timer(const tk_opts *o, hipStream_t s_) : on(o->timing != 0 || o->trace), s(s_), tr(o->trace) {}
    ~Timer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    void reserve_pair(int k, int mode, int prec) {
        if (used + 2 > ev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                (void)hipEventCreate(&e);
                ev.push_back(e);
            }
        }
        tag.resize(used / 2 + 1);
        tag[used / 2] = Tag{k, mode, prec};
    }
    // begin / end pairs may enclose kernel() pairs and other begin / end
    // pairs (a phase around the launches it times)
    std::vector<size_t> open;
    void begin(int k, int mode = -1, int prec = -1) {
        if (!on) return;
        reserve_pair(k, mode, prec);
        (void)hipEventRecord(ev[used], s);
        open.push_back(used);
        used += 2;
    }
    void end() {
        if (!on || open.empty()) return;
        (void)hipEventRecord(ev[open.back() + 1], s);
        open.pop_back();
    }
    // A pair for a single kernel that records them itself at its start and
    // end (kernel time without the dispatch gap an event bracket includes).
    KernelEvents kernel(int k, int mode = -1, int prec = -1) {
        if (!on) return KernelEvents();
        reserve_pair(k, mode, prec);
        const KernelEvents ke{ev[used], ev[used + 1]};
        used += 2;
        return ke;
    }
    // call after a stream synchronisation
    void collect() {
        if (!on) return;
        double ttmc = 0.0;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float t = 0;
            (void)hipEventElapsedTime(&t, ev[i], ev[i + 1]);
            const Tag &g = tag[i / 2];
            ms[g.kind] += t;
            calls[g.kind] += 1;
            if (g.kind == kProj || g.kind == kTtmc) ttmc += t;
            if (tr && tr->events) {
                if (tr->count < tr->capacity)
                    tr->events[tr->count++] = tk_event{g.kind, g.mode, g.prec, sweeps + 1, (double)t};
                else
                    tr->dropped++;
            }
        }
        if (sweeps < 64) sweep_ttmc[sweeps] = ttmc;
        ++sweeps;
        used = 0;
    }
    void report(tk_stats *st) const {
        if (!st) return;
        st->project_ms = ms[kProj];
        st->project_calls = calls[kProj];
        st->ttmc_ms = ms[kProj] + ms[kTtmc];
        st->gram_ms = ms[kGram];
        st->gram_calls = calls[kGram];
        st->eig_ms = ms[kEig];
        st->core_ms = ms[kCore];
        for (int t = 0; t < 64; ++t) st->ttmc_sweep_ms[t] = t < sweeps ? sweep_ttmc[t] : 0.0;
    }
};

}  // namespace tk
