// selector.cpp -- learned plan selector (host side).
#include "selector.h"

#include "../../include/offt.h"

namespace offt {

int learned_choice(int dtype, const int64_t dims[3], int64_t batch, const char* weights_path,
                   PlanChoice* c, std::string* why) {
    (void)dtype; (void)dims; (void)batch; (void)c;
    if (!weights_path) { *why = "no weights"; return OFFT_ERR_IO; }
    *why = "selector not available";
    return OFFT_ERR_IO;
}

}  // namespace offt
