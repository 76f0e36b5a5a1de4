// tune.hip -- autotuner (placeholder until the timing search is in place).
#include "plan.hpp"

namespace mifft {
int tune_plan(Plan&) { return MIFFT_OK; }
} // namespace mifft
