// plan_impl.h -- the plan object behind offt_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/offt.h"
#include "offt_internal.h"

namespace offt {
struct ManyState;
struct DistState;
}

struct offt_plan_s {
    int kind = 0;                 // 1: one grid shape (+batch), 2: uneven batch, 3: 4-D / 5-D grids,
                                  // 4: the distributed flow over virtual processes
    int dtype = 0;
    int64_t dims[3] = {1, 1, 1};
    int64_t batch = 1;
    int normalize = 0;
    offt::PlanChoice choice{};
    offt::PassPlan passes[offt::kMaxDims]{};
    int npass = 0;
    // kind 3: the grid's axes and the plan over them
    int ndim = 3;
    int64_t nd_dims[offt::kMaxDims] = {1, 1, 1, 1, 1};
    offt::NdChoice ndc{};
    // OFFT_LAYOUT_REVERSED: the backward transform reads cba grids, so it is
    // planned as a transform of the reversed shape (Nc, Nb, Na) whose output
    // is reversed back to abc; both directions route through `work` (one
    // batch of grids) where a transposing pass needs it
    int layout = OFFT_LAYOUT_NATURAL;
    offt::PlanChoice choice_b{};
    offt::PassPlan passes_b[3]{};
    void* work = nullptr;
    std::map<int, void*> tw;      // twiddle table per pass length
    std::vector<void*> allocs;    // every device allocation owned by the plan
    std::vector<size_t> alloc_bytes;
    std::string tune_log;         // how the plan was chosen (for describe)
    offt::ManyState* many = nullptr;
    offt::DistState* dist = nullptr;   // kind 4: Np virtual processes
    // use_graph: the passes replayed from HIP graphs captured on `cap`, one
    // per direction ([0] forward, [1] backward)
    int use_graph = 0;
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    const void* g_in[2] = {nullptr, nullptr};   // buffers each instantiated graph holds
    void* g_out[2] = {nullptr, nullptr};

    int64_t workspace_bytes() const;
    int64_t grid_elems() const;   // points of one grid
};

namespace offt {

int check_device();
int validate_dims(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch);
int attach_twiddles(offt_plan_s* p, PassPlan* passes, int npass, hipStream_t s);
int set_choice(offt_plan_s* p, const PlanChoice& c, hipStream_t s);
int set_choice_b(offt_plan_s* p, const PlanChoice& c, hipStream_t s);
// The passes a direction runs (the backward list differs for reversed layouts).
const PassPlan* dir_passes(const offt_plan_s* p, int dir);
void reversed_dims(const int64_t dims[3], int64_t out[3]);
// normalize: -1 the plan's normalize_inverse, else 0 / 1 for this call.
// Passes [i0, i1) of the list (i1 < 0: to the end) as the whole transform
// runs them: buffers, conjugation and scaling by their place in the list, a
// slab schedule's passes interleaved slab by slab.
int exec_passes(const offt_plan_s* p, const PassPlan* passes, int npass, const void* in, void* out,
                void* work, int dir, hipStream_t s, int normalize = -1, int i0 = 0, int i1 = -1);
void free_plan(offt_plan_s* p);

// Tuning (tuner.cpp): fills *choice for EXHAUSTIVE / LEARNED modes.
// For reversed layouts also *choice_b (the backward plan on the reversed shape).
int select_plan(offt_plan_s* p, const offt_opts& o, PlanChoice* choice, PlanChoice* choice_b);
// The same for kind-3 plans (EXHAUSTIVE; LEARNED falls back to it).
int select_plan_nd(offt_plan_s* p, const offt_opts& o, NdChoice* choice);
std::string describe_plan(const offt_plan_s* p);

// Uneven batches (many.hip).
void release_many(offt_plan_s* p);
std::string describe_many(const offt_plan_s* p);

// The distributed flow over virtual processes (dist.hip): the first `steps`
// of the five steps, method < 0 the plan's, normalize < 0 the plan's.
void release_dist(offt_plan_s* p);
std::string describe_dist(const offt_plan_s* p);
int exec_dist(const offt_plan_s* p, int dir, int steps, const void* in, void* out, int method, int normalize,
              hipStream_t s);

}  // namespace offt
