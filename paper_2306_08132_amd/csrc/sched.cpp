// Serving loop of the grasp library (continuous batching). Placeholder until
// the scheduler lands: shutting a context down has nothing to stop.
#include "context.h"

namespace grasp {
struct Scheduler {};
}  // namespace grasp

extern "C" void grasp_shutdown_scheduler(grasp_ctx* ctx) { (void)ctx; }
