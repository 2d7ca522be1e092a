// Internal hooks of the schedule selector (see selector.cpp).
#pragma once
#include "../../include/lu.h"

namespace lu {
bool selector_enabled();
int selector_predict(int n, int prec, lu_schedule_t* out);   // 0 = predicted, 1 = default used
}  // namespace lu
