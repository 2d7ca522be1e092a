// Internal view of the look-ahead task list (see include/lu_plan.h).
#pragma once
#include <vector>

#include "../../include/lu_plan.h"

namespace lu {

enum { kTaskPanel = LU_TASK_PANEL, kTaskUpdate = LU_TASK_UPDATE, kTaskLswap = LU_TASK_LSWAP };
constexpr int kPlanStreams = LU_PLAN_STREAMS;

struct PlanTask {
    int kind, step, col_begin, col_end, stream;
    int nwait;
    int wait[LU_PLAN_MAX_WAIT];
    int record;
};

int build_plan(int n, int b, int depth, std::vector<PlanTask>& out);

}  // namespace lu
