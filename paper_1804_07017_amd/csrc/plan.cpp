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
#include <cstdlib>

namespace lu {

namespace {

struct Access {
    int w0, w1;      // columns written
    int r0, r1;      // columns read (besides the written ones)
    int ipiv_w;      // pivot block written (-1 none)
    int ipiv_r;      // pivot block read (-1 none, -2 every block)
};

inline bool overlap(int a0, int a1, int b0, int b1) { return a0 < b1 && b0 < a1 && a0 < a1 && b0 < b1; }

Access access_of(const PlanTask& t, const std::vector<int>& starts) {
    Access a{t.col_begin, t.col_end, 0, 0, -1, -1};
    switch (t.kind) {
    case kTaskPanel:
        a.ipiv_w = t.step;
        break;
    case kTaskUpdate: {
        a.r0 = starts[t.step]; a.r1 = starts[t.step + 1];   // reads the factored panel k (L11, L21)
        a.ipiv_r = t.step;
        break;
    }
    case kTaskLswap:
        a.ipiv_r = t.step;
        break;
    case kTaskLperm:
        a.ipiv_r = -2;
        break;
    }
    return a;
}

bool conflicts(const Access& e, const Access& l) {
    // e is earlier in program order, l later
    if (overlap(e.w0, e.w1, l.w0, l.w1)) return true;   // WAW
    if (overlap(e.w0, e.w1, l.r0, l.r1)) return true;   // RAW
    if (overlap(e.r0, e.r1, l.w0, l.w1)) return true;   // WAR
    if (e.ipiv_w >= 0 && (e.ipiv_w == l.ipiv_r || l.ipiv_r == -2 || e.ipiv_w == l.ipiv_w)) return true;
    if (l.ipiv_w >= 0 && (e.ipiv_r == l.ipiv_w || e.ipiv_r == -2)) return true;
    return false;
}

}  // namespace

// Trailing size at or below which panels are at most 256 wide (the middle
// tier of the taper; 0: no middle tier).  LU_TAPER_MID overrides it.
int taper_mid(int prec) {
    static const int env = [] {
        const char* e = std::getenv("LU_TAPER_MID");
        return (e && *e) ? std::atoi(e) : -1;
    }();
    if (env >= 0) return env;
    return prec == 0 ? kTaperMid64 : kTaperMid32;
}

// Trailing size at or below which panels are 128 wide; LU_TAPER_NARROW
// overrides it for every precision.
int taper_narrow(int prec) {
    static const int env = [] {
        const char* e = std::getenv("LU_TAPER_NARROW");
        return (e && *e) ? std::atoi(e) : -1;
    }();
    if (env >= 0) return env;
    return prec == 0 ? kTaperNarrow64 : kTaperNarrow32;
}

int taper_width(int prec, int trailing) {
    // Early termination, done statically: the panel narrows as the trailing
    // matrix shrinks, so that in the tail the factorization of the next panel
    // stays short next to the update it overlaps.  The widths are the block
    // sizes that are fastest for a whole factorization of that size on this
    // GPU (the schedule sweep), per precision class.
    const int t128 = taper_narrow(prec);
    if (trailing <= t128) return 128;
    if (trailing <= taper_mid(prec)) return 256;
    return 1 << 30;
}

std::vector<int> panel_starts(int n, int b, int taper, int prec) {
    std::vector<int> st;
    if (n <= 0 || b < 1) return st;
    int c = 0;
    st.push_back(0);
    while (c < n) {
        int w = b;
        if (taper > 0) w = std::min(w, taper_width(prec, n - c));
        c = std::min(n, c + w);
        st.push_back(c);
    }
    return st;
}

int build_plan(int n, int b, int depth, std::vector<PlanTask>& out) {
    out.clear();
    if (n < 0) return -1;
    if (b < 1) return -2;
    if (depth < 0 || depth > 2) return -3;
    return build_plan(n, panel_starts(n, b, 0, 0), depth, out);
}

int build_plan(int n, const std::vector<int>& starts, int depth, std::vector<PlanTask>& out, int swaps) {
    const bool lswap = swaps == 1;
    out.clear();
    if (n < 0) return -1;
    if (depth < 0 || depth > 2) return -3;
    if (n == 0) return 0;
    const int N = (int)starts.size() - 1;
    if (N < 1 || starts[0] != 0 || starts[N] != n) return -4;
    for (int j = 0; j < N; ++j)
        if (starts[j + 1] <= starts[j]) return -4;
    auto panel_cols = [&](int j, int& c0, int& c1) { c0 = starts[j]; c1 = starts[j + 1]; };
    auto col_of = [&](int j) { return j >= N ? n : starts[j]; };   // first column of panel j (n past the end)
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
            if (k >= 1 && lswap) push(kTaskLswap, k, 0, c0, 0);
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
            push(kTaskUpdate, k, col_of(k + d + 1), n, 0);                            // TU_k, right part
            if (j < N) {
                panel_cols(j, c0, c1);
                for (int i = k + 1; i < j; ++i) push(kTaskUpdate, i, c0, c1, 1);
                push(kTaskPanel, j, c0, c1, 1);
            }
            if (k >= 1 && lswap) push(kTaskLswap, k, 0, starts[k], 2);
        }
    }
    // deferred left interchanges: one task after everything else, on the update stream
    if (swaps == 2 && N >= 2) push(kTaskLperm, N - 1, 0, starts[N - 1], 0);
    // Derive cross-stream waits from data accesses.
    const int T = (int)out.size();
    std::vector<Access> acc(T);
    for (int i = 0; i < T; ++i) acc[i] = access_of(out[i], starts);
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

namespace {

int export_plan(const std::vector<lu::PlanTask>& v, lu_plan_task_t* out, int max_tasks) {
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

}  // namespace

extern "C" int lu_plan_build(int n, int b, int depth, lu_plan_task_t* out, int max_tasks) {
    std::vector<lu::PlanTask> v;
    int r = lu::build_plan(n, b, depth, v);
    if (r < 0) return r;
    return export_plan(v, out, max_tasks);
}

extern "C" int lu_plan_panels(int n, int b, int taper, int prec, int* starts, int max_starts) {
    if (n < 0) return -1;
    if (b < 1) return -2;
    if (prec < 0 || prec > 3) return -4;
    if (n == 0) return 0;
    const std::vector<int> st = lu::panel_starts(n, b, taper, prec);
    const int N = (int)st.size() - 1;
    if (!starts || max_starts < N + 1) return -5;
    for (int j = 0; j <= N; ++j) starts[j] = st[j];
    return N;
}

extern "C" int lu_plan_build_panels_ex(int n, const int* starts, int npanels, int depth, int interchanges,
                                       lu_plan_task_t* out, int max_tasks) {
    if (n < 0) return -1;
    if (n > 0 && (!starts || npanels < 1)) return -4;
    std::vector<int> st;
    if (n > 0) st.assign(starts, starts + npanels + 1);
    if (interchanges < 0 || interchanges > 2) return -6;
    std::vector<lu::PlanTask> v;
    int r = lu::build_plan(n, st, depth, v, interchanges);
    if (r < 0) return r;
    return export_plan(v, out, max_tasks);
}

extern "C" int lu_plan_build_panels(int n, const int* starts, int npanels, int depth, lu_plan_task_t* out,
                                    int max_tasks) {
    if (n < 0) return -1;
    if (n > 0 && (!starts || npanels < 1)) return -4;
    std::vector<int> st;
    if (n > 0) st.assign(starts, starts + npanels + 1);
    std::vector<lu::PlanTask> v;
    int r = lu::build_plan(n, st, depth, v);
    if (r < 0) return r;
    return export_plan(v, out, max_tasks);
}
