// selector.cpp -- learned plan selector (host side).
//
// The paper tunes the communication method at run time by executing every
// candidate (Sec. 3.2.3) and notes that model-driven selection suits
// single-node tuning.  Here a small network, trained on timings the
// exhaustive tuner produced, predicts ln(time) of each candidate plan from
// plan_features(); the argmin is chosen without timing anything.  Weights
// file (text):
//   offt-selector 1
//   dims <D> <H>
//   mean <D floats>      feature standardisation
//   std <D floats>
//   target <mean> <std>  standardisation of ln(time in ms)
//   params <P> <P floats>
#include "selector.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

#include "../../include/offt.h"
#include "plan_impl.h"

namespace offt {

static const int kOrders[6][3] = {{2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 0, 2}, {0, 2, 1}, {0, 1, 2}};

std::vector<PlanChoice> selector_candidates(int dtype, const int64_t dims[3], int64_t batch) {
    std::vector<PlanChoice> out = candidate_choices(dtype, dims);
    if (out.empty()) return out;
    // the heuristic with one axis's access mode switched (streaming <->
    // cached grid data; by default the mode follows the grid's size)
    const PlanChoice base = out[0];
    const int64_t bytes = dims[0] * dims[1] * dims[2] * batch * (int64_t)elem_size(dtype);
    for (int ax = 0; ax < 3; ++ax) {
        if (dims[ax] <= 1 || !base.k[ax]) continue;
        PlanChoice c = base;
        c.io[ax] = resolve_stream(base.io[ax], bytes) ? kIoCached : kIoStream;
        out.push_back(c);
    }
    return out;
}

void plan_features(int dtype, const int64_t dims[3], int64_t batch, const PlanChoice& c, float* f) {
    for (int i = 0; i < kFeatureDim; ++i) f[i] = 0.f;
    const double N = (double)dims[0] * (double)dims[1] * (double)dims[2];
    for (int ax = 0; ax < 3; ++ax) f[ax] = (float)std::log2((double)dims[ax]);
    f[3] = (float)std::log2((double)batch);
    f[4] = dtype == OFFT_C2C_F32 ? 1.f : 0.f;
    f[5] = (float)std::log2(N * (double)batch);
    for (int o = 0; o < 6; ++o)
        if (c.order[0] == kOrders[o][0] && c.order[1] == kOrders[o][1] && c.order[2] == kOrders[o][2]) f[6 + o] = 1.f;
    int pos[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) pos[c.order[i]] = i;
    for (int ax = 0; ax < 3; ++ax) {
        float* g = f + 12 + kAxisFeatures * ax;
        const KernelEntry* k = c.k[ax];
        if (dims[ax] <= 1 || !k) continue;
        int64_t m2 = 1;
        for (int j = ax + 1; j < 3; ++j) m2 *= dims[j];
        g[0] = m2 > 1 ? 1.f : 0.f;
        g[1] = (float)k->nstages;
        for (int s = 0; s < k->nstages; ++s) {
            switch (k->radices[s]) {
                case 32: g[11] += 1.f; break;
                case 16: g[2] += 1.f; break;
                case 8: g[3] += 1.f; break;
                case 4: g[4] += 1.f; break;
                case 2: g[5] += 1.f; break;
                case 3: g[6] += 1.f; break;
                case 5: g[7] += 1.f; break;
                default: break;
            }
        }
        g[8] = (float)c.logW[ax];
        g[9] = (float)std::log2((double)k->tpl);
        g[10] = (float)pos[ax] * 0.5f;
        g[12] = (float)std::log2((double)k->nparts);
        g[13] = (float)c.xcd[ax];
        // the access mode the pass runs with (streaming or cached grid data)
        g[14] = (float)resolve_stream(c.io[ax], (int64_t)(N * (double)batch) * (int64_t)elem_size(dtype));
    }
}

struct Weights {
    int D = 0, H = 0;
    std::vector<float> mean, stdv, params;
    float tmean = 0.f, tstd = 1.f;
};

static bool read_floats(std::istream& is, int n, std::vector<float>* v) {
    v->resize(n);
    for (int i = 0; i < n; ++i)
        if (!(is >> (*v)[i]) || !std::isfinite((*v)[i])) return false;
    return true;
}

static bool load_weights(const char* path, Weights* w, std::string* why) {
    std::ifstream f(path);
    if (!f) { *why = "weights file unreadable"; return false; }
    std::string tag;
    int ver = 0;
    if (!(f >> tag >> ver) || tag != "offt-selector" || ver != 1) { *why = "not a selector weights file"; return false; }
    if (!(f >> tag >> w->D >> w->H) || tag != "dims" || w->D != kFeatureDim || w->H < 1 || w->H > 256) {
        *why = "weights do not match the feature layout";
        return false;
    }
    int64_t P = 0;
    if (!(f >> tag) || tag != "mean" || !read_floats(f, w->D, &w->mean) || !(f >> tag) || tag != "std" ||
        !read_floats(f, w->D, &w->stdv) || !(f >> tag >> w->tmean >> w->tstd) || tag != "target" ||
        !(f >> tag >> P) || tag != "params" || P != offt_mlp_nparams(w->D, w->H) ||
        !read_floats(f, (int)P, &w->params)) {
        *why = "weights file corrupt";
        return false;
    }
    for (float s : w->stdv)
        if (!(s > 0.f)) { *why = "weights file corrupt"; return false; }
    return true;
}

// Host forward pass of the network (same arithmetic as the GPU kernel).
static float forward(const Weights& w, const float* x) {
    const int D = w.D, H = w.H;
    const float* W1 = w.params.data();
    const float* b1 = W1 + (size_t)H * D;
    const float* W2 = b1 + H;
    const float* b2 = W2 + (size_t)H * H;
    const float* w3 = b2 + H;
    const float* b3 = w3 + H;
    std::vector<float> a1(H), a2(H);
    for (int j = 0; j < H; ++j) {
        float s = b1[j];
        for (int k = 0; k < D; ++k) s += W1[(size_t)j * D + k] * x[k];
        a1[j] = s > 0.f ? s : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        float s = b2[j];
        for (int i = 0; i < H; ++i) s += W2[(size_t)j * H + i] * a1[i];
        a2[j] = s > 0.f ? s : 0.f;
    }
    float y = b3[0];
    for (int i = 0; i < H; ++i) y += w3[i] * a2[i];
    return y;
}

int learned_choice(int dtype, const int64_t dims[3], int64_t batch, const char* weights_path, PlanChoice* c,
                   std::string* why) {
    if (!weights_path) { *why = "no weights"; return OFFT_ERR_IO; }
    static std::mutex mu;
    static std::map<std::string, Weights> cache;
    Weights w;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(weights_path);
        if (it == cache.end()) {
            if (!load_weights(weights_path, &w, why)) return OFFT_ERR_IO;
            it = cache.emplace(weights_path, w).first;
        }
        w = it->second;
    }
    const std::vector<PlanChoice> cands = selector_candidates(dtype, dims, batch);
    if (cands.empty()) { *why = "no candidate plans"; return OFFT_ERR_UNSUPPORTED_SIZE; }
    std::vector<float> x(kFeatureDim);
    int best = -1;
    float best_y = 0.f;
    for (size_t i = 0; i < cands.size(); ++i) {
        plan_features(dtype, dims, batch, cands[i], x.data());
        for (int k = 0; k < kFeatureDim; ++k) x[k] = (x[k] - w.mean[k]) / w.stdv[k];
        const float y = forward(w, x.data());
        if (!std::isfinite(y)) continue;
        if (best < 0 || y < best_y) { best = (int)i; best_y = y; }
    }
    if (best < 0) { *why = "no finite prediction"; return OFFT_ERR_IO; }
    *c = cands[best];
    return OFFT_SUCCESS;
}

}  // namespace offt

using namespace offt;

extern "C" {

int offt_feature_dim(void) { return kFeatureDim; }

int offt_candidates(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, char* plans, size_t plans_bytes,
                    float* features, int max) {
    const int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const int64_t dims[3] = {Na, Nb, Nc};
    const std::vector<PlanChoice> cands = selector_candidates(dtype, dims, batch);
    const int n = (int)cands.size();
    if (max < 0 || (max > 0 && (!plans || !features))) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
    size_t pos = 0;
    for (int i = 0; i < std::min(n, max); ++i) {
        plan_features(dtype, dims, batch, cands[i], features + (size_t)i * kFeatureDim);
        const std::string s = choice_to_string(cands[i], dims);
        if (pos + s.size() + 1 > plans_bytes) { set_error(OFFT_ERR_INVALID_ARG); return OFFT_ERR_INVALID_ARG; }
        memcpy(plans + pos, s.c_str(), s.size() + 1);
        pos += s.size() + 1;
    }
    set_error(OFFT_SUCCESS);
    return n;
}

int offt_plan_features(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, const char* plan, float* out) {
    int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc == OFFT_SUCCESS && (!plan || !out)) rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const int64_t dims[3] = {Na, Nb, Nc};
    PlanChoice c;
    if (!choice_from_string(plan, dtype, dims, &c, false)) { set_error(OFFT_ERR_BAD_PLAN); return OFFT_ERR_BAD_PLAN; }
    plan_features(dtype, dims, batch, c, out);
    set_error(OFFT_SUCCESS);
    return OFFT_SUCCESS;
}

int offt_selector_scores(const char* weights_path, const float* features, int n, float* scores) {
    if (!weights_path || n < 0 || (n > 0 && (!features || !scores))) {
        set_error(OFFT_ERR_INVALID_ARG);
        return OFFT_ERR_INVALID_ARG;
    }
    Weights w;
    std::string why;
    if (!load_weights(weights_path, &w, &why)) { set_error(OFFT_ERR_IO); return OFFT_ERR_IO; }
    std::vector<float> x(kFeatureDim);
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < kFeatureDim; ++k) x[k] = (features[(size_t)i * kFeatureDim + k] - w.mean[k]) / w.stdv[k];
        scores[i] = forward(w, x.data()) * w.tstd + w.tmean;
    }
    set_error(OFFT_SUCCESS);
    return OFFT_SUCCESS;
}

int offt_selector_choose(int64_t Na, int64_t Nb, int64_t Nc, int dtype, int64_t batch, const char* weights_path,
                         char* buf, size_t n) {
    int rc = validate_dims(Na, Nb, Nc, dtype, batch);
    if (rc == OFFT_SUCCESS && (!weights_path || (!buf && n))) rc = OFFT_ERR_INVALID_ARG;
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const int64_t dims[3] = {Na, Nb, Nc};
    PlanChoice c;
    std::string why;
    rc = learned_choice(dtype, dims, batch, weights_path, &c, &why);
    if (rc != OFFT_SUCCESS) { set_error(rc); return rc; }
    const std::string s = choice_to_string(c, dims);
    if (n) {
        const size_t m = std::min(n - 1, s.size());
        memcpy(buf, s.data(), m);
        buf[m] = 0;
    }
    set_error(OFFT_SUCCESS);
    return (int)s.size();
}

}  // extern "C"
