// Plan log on stderr, switched on by the environment variable LFFT_LOG
// (any value but "0"): the schedule of every plan the C ABI creates.
#pragma once
#include "plan.hpp"

namespace lfft {

struct BatchPlan;

bool plan_log_on();
void log_lattice_plan(const LatticePlan* p, const char* label);
void log_wave_plan(const WavePlan* w);
void log_batch_plan(const BatchPlan* b, const char* label);

}  // namespace lfft
