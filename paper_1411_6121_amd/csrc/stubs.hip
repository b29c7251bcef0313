// entry points not built yet
#include "ctx.hpp"
extern "C" int dugks_batch_create(const dugks_config*, int, const int64_t*, void*, dugks_batch** out)
{ if (out) *out = nullptr; return DUGKS_EUNSUPPORTED; }
extern "C" int dugks_batch_init(dugks_batch*, void*, void*) { return DUGKS_EUNSUPPORTED; }
extern "C" int dugks_batch_run(dugks_batch*, void*, void*, const void*, const int64_t*, double, int, int, void*, int*)
{ return DUGKS_EUNSUPPORTED; }
extern "C" void dugks_batch_destroy(dugks_batch*) {}
extern "C" const char* dugks_batch_last_error(const dugks_batch*) { return "batch not built yet"; }
