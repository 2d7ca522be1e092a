// Internal view of the look-ahead task list (see include/lu_plan.h).
#pragma once
#include <vector>

#include "../../include/lu_plan.h"

namespace lu {

enum { kTaskPanel = LU_TASK_PANEL, kTaskUpdate = LU_TASK_UPDATE, kTaskLswap = LU_TASK_LSWAP, kTaskLperm = LU_TASK_LPERM };
constexpr int kPlanStreams = LU_PLAN_STREAMS;

struct PlanTask {
    int kind, step, col_begin, col_end, stream;
    int nwait;
    int wait[LU_PLAN_MAX_WAIT];
    int record;
};

// Panel boundaries: starts[0] = 0 < starts[1] < ... < starts[N] = n.
// taper <= 0: every panel b wide (the last one ragged); taper > 0: the width
// of panel j is min(b, taper_width(prec, n - starts[j])).
std::vector<int> panel_starts(int n, int b, int taper, int prec);
int taper_width(int prec, int trailing);
// middle tier of the taper: panels at most 256 wide while the trailing size is
// in (the 128 threshold, taper_mid]; 0 = none
constexpr int kTaperMid64 = 0, kTaperMid32 = 0;
int taper_mid(int prec);
// trailing size at or below which panels are 128 wide: FP64, FP32 and mixed
constexpr int kTaperNarrow64 = 12288, kTaperNarrow32 = 16384;
int taper_narrow(int prec);

int build_plan(int n, int b, int depth, std::vector<PlanTask>& out);
// swaps: 0 no left interchanges (a factorization without row interchanges),
// 1 one LSWAP task per step, 2 one LPERM task at the end
int build_plan(int n, const std::vector<int>& starts, int depth, std::vector<PlanTask>& out, int swaps = 1);

}  // namespace lu
