// Look-ahead schedule: the task DAG of the blocked right-looking LU and its
// placement on streams (paper Sec. 3.3 Listing 3, Sec. 4 Listing 5): stream 0
// runs the bulk trailing update, stream 1 the look-ahead panel work, stream 2
// the interchanges of finished columns left of each panel (off the critical
// path; nothing reads those columns again before the end).
//
// The program order built here is itself a valid sequential order of the
// algorithm; stream placement only adds concurrency.  Cross-stream waits are
// derived from the data each task touches (column ranges and pivot blocks),
// never written by hand, so two tasks that may run at the same time never
// touch the same columns.
#include "plan.hpp"

#include <algorithm>

namespace lu {

namespace {

struct Access {
    int w0, w1;      // columns written
    int r0, r1;      // columns read (besides the written ones)
    int ipiv_w;      // pivot block written (-1 none)
    int ipiv_r;      // pivot block read (-1 none)
};

inline bool overlap(int a0, int a1, int b0, int b1) { return a0 < b1 && b0 < a1 && a0 < a1 && b0 < b1; }

Access access_of(const PlanTask& t, int b, int n) {
    Access a{t.col_begin, t.col_end, 0, 0, -1, -1};
    switch (t.kind) {
    case kTaskPanel:
        a.ipiv_w = t.step;
        break;
    case kTaskUpdate: {
        int p0 = t.step * b, p1 = std::min(n, p0 + b);
        a.r0 = p0; a.r1 = p1;          // reads the factored panel k (L11, L21)
        a.ipiv_r = t.step;
        break;
    }
    case kTaskLswap:
        a.ipiv_r = t.step;
        break;
    }
    return a;
}

bool conflicts(const Access& e, const Access& l) {
    // e is earlier in program order, l later
    if (overlap(e.w0, e.w1, l.w0, l.w1)) return true;   // WAW
    if (overlap(e.w0, e.w1, l.r0, l.r1)) return true;   // RAW
    if (overlap(e.r0, e.r1, l.w0, l.w1)) return true;   // WAR
    if (e.ipiv_w >= 0 && (e.ipiv_w == l.ipiv_r || e.ipiv_w == l.ipiv_w)) return true;
    if (l.ipiv_w >= 0 && e.ipiv_r == l.ipiv_w) return true;
    return false;
}

}  // namespace

int build_plan(int n, int b, int depth, std::vector<PlanTask>& out) {
    out.clear();
    if (n < 0) return -1;
    if (b < 1) return -2;
    if (depth < 0 || depth > 2) return -3;
    if (n == 0) return 0;
    const int N = (n + b - 1) / b;
    auto panel_cols = [&](int j, int& c0, int& c1) { c0 = j * b; c1 = std::min(n, c0 + b); };
    auto push = [&](int kind, int step, int c0, int c1, int stream) {
        if (c0 >= c1) return;
        PlanTask t{};
        t.kind = kind; t.step = step; t.col_begin = c0; t.col_end = c1; t.stream = stream;
        out.push_back(t);
    };
    int c0, c1;
    if (depth == 0) {
        // Listing 3: PF(k); TU(k) on one stream.
        for (int k = 0; k < N; ++k) {
            panel_cols(k, c0, c1);
            push(kTaskPanel, k, c0, c1, 0);
            push(kTaskUpdate, k, c1, n, 0);
            if (k >= 1) push(kTaskLswap, k, 0, k * b, 0);
        }
    } else {
        const int d = depth;
        panel_cols(0, c0, c1);
        push(kTaskPanel, 0, c0, c1, 1);
        // prologue: panels 1..d-1 are brought up to date and factored ahead
        for (int j = 1; j <= std::min(d - 1, N - 1); ++j) {
            panel_cols(j, c0, c1);
            for (int i = 0; i < j; ++i) push(kTaskUpdate, i, c0, c1, 1);
            push(kTaskPanel, j, c0, c1, 1);
        }
        for (int k = 0; k < N; ++k) {
            const int j = k + d;                         // panel factored during step k's bulk update
            if (j < N) { panel_cols(j, c0, c1); push(kTaskUpdate, k, c0, c1, 0); }   // TU_k, left part
            push(kTaskUpdate, k, std::min(n, (k + d + 1) * b), n, 0);                 // TU_k, right part
            if (j < N) {
                panel_cols(j, c0, c1);
                for (int i = k + 1; i < j; ++i) push(kTaskUpdate, i, c0, c1, 1);
                push(kTaskPanel, j, c0, c1, 1);
            }
            if (k >= 1) push(kTaskLswap, k, 0, k * b, 2);
        }
    }
    // Derive cross-stream waits from data accesses.
    const int T = (int)out.size();
    std::vector<Access> acc(T);
    for (int i = 0; i < T; ++i) acc[i] = access_of(out[i], b, n);
    // covered[s][u]: latest task of stream u that stream s already waits for
    int covered[kPlanStreams][kPlanStreams];
    for (auto& r : covered) for (int& c : r) c = -1;
    for (int i = 0; i < T; ++i) {
        PlanTask& t = out[i];
        const int s = t.stream;
        for (int u = 0; u < kPlanStreams; ++u) {
            if (u == s) continue;
            int need = -1;
            for (int e = i - 1; e > covered[s][u]; --e) {
                if (out[e].stream != u) continue;
                if (conflicts(acc[e], acc[i])) { need = e; break; }
            }
            if (need >= 0) {
                t.wait[t.nwait++] = need;
                out[need].record = 1;
                covered[s][u] = need;
            }
        }
    }
    return T;
}

}  // namespace lu

extern "C" int lu_plan_build(int n, int b, int depth, lu_plan_task_t* out, int max_tasks) {
    std::vector<lu::PlanTask> v;
    int r = lu::build_plan(n, b, depth, v);
    if (r < 0) return r;
    if ((int)v.size() > max_tasks) return -5;
    for (size_t i = 0; i < v.size(); ++i) {
        lu_plan_task_t& o = out[i];
        o.kind = v[i].kind; o.step = v[i].step;
        o.col_begin = v[i].col_begin; o.col_end = v[i].col_end;
        o.stream = v[i].stream; o.nwait = v[i].nwait;
        for (int w = 0; w < LU_PLAN_MAX_WAIT; ++w) o.wait[w] = w < v[i].nwait ? v[i].wait[w] : -1;
        o.record = v[i].record;
    }
    return (int)v.size();
}
