// many.hip -- uneven batches of grids.
#include "../../include/offt.h"
#include "offt_internal.h"
#include "plan_impl.h"

namespace offt {

void release_many(offt_plan_s* p) { (void)p; }
std::string describe_many(const offt_plan_s* p) { (void)p; return "many"; }

}  // namespace offt

extern "C" {

offt_plan_t offt_plan_many(int count, const int64_t* dims, int dtype, const offt_opts* o) {
    (void)count; (void)dims; (void)dtype; (void)o;
    offt::set_error(OFFT_ERR_INVALID_ARG);
    return nullptr;
}

int64_t offt_many_offset(offt_plan_t p, int i) {
    (void)p; (void)i;
    offt::set_error(OFFT_ERR_BAD_PLAN);
    return OFFT_ERR_BAD_PLAN;
}

int offt_exec_many(offt_plan_t p, const void* in, void* out, int direction, int use_graph, void* stream) {
    (void)p; (void)in; (void)out; (void)direction; (void)use_graph; (void)stream;
    offt::set_error(OFFT_ERR_BAD_PLAN);
    return OFFT_ERR_BAD_PLAN;
}

}  // extern "C"
