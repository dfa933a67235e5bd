// Opaque handle types of the C ABI (include/lfft.h): each wraps one host plan.
#pragma once

#include "batch.hpp"
#include "plan.hpp"

struct lfft_plan_s {
  lfft::LatticePlan* p;
};
struct lwt_plan_s {
  lfft::WavePlan* w;
};
struct lfft_batch_s {
  lfft::BatchPlan* b;
};
