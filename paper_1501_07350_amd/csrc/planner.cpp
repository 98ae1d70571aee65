// planner.cpp -- kernel registry lookup, heuristic plan, candidate plans for
// tuning, plan strings, and the [M1][L][M2] pass descriptors of a plan.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <tuple>

#include "offt_internal.h"
#include "../../include/offt.h"

namespace offt {

#include "_gen/registry_parts.inc"

namespace {
struct Table {
    const KernelEntry* p;
    int n;
};
}  // namespace

const std::vector<const KernelEntry*>& registry() {
    static const std::vector<const KernelEntry*> all = [] {
        std::vector<const KernelEntry*> v;
        const Table tables[] = {OFFT_REGISTRY_TABLES};
        for (const Table& t : tables)
            for (int i = 0; i < t.n; ++i) v.push_back(&t.p[i]);
        return v;
    }();
    return all;
}

// Kernels of one length, default first: radix <= 16 before radix-32
// sequences, then fewest stages, then largest leading radix, then the most
// threads per line (one butterfly of the largest radix per thread), then
// whole-line exchanges before exchanges in parts.
std::vector<const KernelEntry*> kernels_for(int dtype, int L) {
    std::vector<const KernelEntry*> v;
    for (const KernelEntry* e : registry())
        if (e->dtype == dtype && e->L == L) v.push_back(e);
    auto key = [](const KernelEntry* e) {
        int maxr = 0;
        for (int i = 0; i < e->nstages; ++i) maxr = std::max(maxr, e->radices[i]);
        return std::make_tuple(maxr > 16, e->nstages, -maxr, -e->tpl, e->nparts);
    };
    std::stable_sort(v.begin(), v.end(),
                     [&](const KernelEntry* x, const KernelEntry* y) { return key(x) < key(y); });
    return v;
}

static int default_tpl(const KernelEntry* k) {
    int maxr = 0;
    for (int i = 0; i < k->nstages; ++i) maxr = std::max(maxr, k->radices[i]);
    return k->L / maxr;
}

size_t elem_size(int dtype) { return dtype == OFFT_C2C_F64 ? 16 : 8; }

bool smooth235(int64_t n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

static int ilog2(int64_t v) {
    int k = 0;
    while ((int64_t(1) << (k + 1)) <= v) ++k;
    return k;
}

int64_t lds_limit() {
    static const int64_t lim = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
            (void)hipGetLastError();
            return int64_t(64 * 1024);
        }
        return int64_t(v);
    }();
    return lim;
}

bool tile_fits(const KernelEntry* k, int logW, int dtype) {
    if (!k || logW < 0) return false;
    const int64_t W = int64_t(1) << logW;
    const int64_t threads = W * k->tpl;
    if (threads > k->max_threads) return false;
    const int64_t lds = tile_lds_elems((int)W, k->L, k->nparts) * (int64_t)elem_size(dtype);
    return lds <= lds_limit();
}

int fit_logW(const KernelEntry* k, int logW, int dtype) {
    if (!k) return 0;
    while (logW > 0 && !tile_fits(k, logW, dtype)) --logW;
    return logW;
}

static int max_radix(const KernelEntry* k) {
    int maxr = 0;
    for (int i = 0; i < k->nstages; ++i) maxr = std::max(maxr, k->radices[i]);
    return maxr;
}

// Heuristic tile width: strided lines get 256-byte row segments (16 columns
// of complex128, 32 of complex64), and radix-32 kernels 32 columns in both
// precisions; contiguous lines ~512 threads per workgroup for complex128 and
// ~128 for complex64.
static int strided_logW(const KernelEntry* k, int dtype) {
    return max_radix(k) >= 32 ? 5 : (dtype == OFFT_C2C_F64 ? 4 : 5);
}

static int default_logW(const KernelEntry* k, int dtype, bool strided) {
    if (!k) return 0;
    int logW;
    if (strided)
        logW = strided_logW(k, dtype);
    else
        logW = ilog2(std::max<int64_t>(1, (dtype == OFFT_C2C_F64 ? 512 : 128) / k->tpl));
    return fit_logW(k, logW, dtype);
}

// Default kernel of an axis: the first in kernels_for() order whose tile at the
// heuristic width fits; contiguous axes take the first kernel with whole-line
// exchanges and radix <= 16.  Strided axes of length >= 512 look first at
// radix-32 kernels whose LDS exchanges run in 2 parts (one exchange per line
// instead of two, half the LDS per tile), then at the other 2-part kernels:
// on MI355X these were the fastest, or within 0.5% of it, for every strided
// pass measured at 512^3 (both precisions) and 1024^3 (complex64).
static const KernelEntry* default_kernel(int dtype, int L, bool strided) {
    std::vector<const KernelEntry*> ks;
    if (strided && L >= 512) {
        for (const KernelEntry* k : kernels_for(dtype, L))
            if (k->nparts == 2 && max_radix(k) >= 32) ks.push_back(k);
        for (const KernelEntry* k : kernels_for(dtype, L))
            if (k->nparts == 2 && max_radix(k) <= 16) ks.push_back(k);
    }
    for (const KernelEntry* k : kernels_for(dtype, L))
        if (k->nparts == 1 && max_radix(k) <= 16) ks.push_back(k);
    if (ks.empty()) return nullptr;
    if (!strided) return ks[0];
    for (const KernelEntry* k : ks)
        if (default_logW(k, dtype, true) >= strided_logW(k, dtype)) return k;
    for (const KernelEntry* k : ks)
        if (k->nparts == 1) return k;
    return ks[0];
}

static bool axis_strided(int axis, const int64_t dims[3]) {
    // M2 of an axis: product of the later axes' lengths
    int64_t m2 = 1;
    for (int j = axis + 1; j < 3; ++j) m2 *= dims[j];
    return m2 > 1;
}

PlanChoice default_choice(int dtype, const int64_t dims[3]) {
    PlanChoice c;
    c.order[0] = 2; c.order[1] = 1; c.order[2] = 0;   // c, then b, then a
    for (int ax = 0; ax < 3; ++ax) {
        c.k[ax] = nullptr;
        c.logW[ax] = 0;
        if (dims[ax] > 1) {
            const bool strided = axis_strided(ax, dims);
            const KernelEntry* k = default_kernel(dtype, (int)dims[ax], strided);
            if (k) {
                c.k[ax] = k;
                c.logW[ax] = default_logW(k, dtype, strided);
            }
        }
    }
    return c;
}

std::vector<PlanChoice> candidate_choices(int dtype, const int64_t dims[3]) {
    std::vector<PlanChoice> out;
    const PlanChoice base = default_choice(dtype, dims);
    out.push_back(base);
    // per-axis variants with the default order: other kernels (radix
    // sequence, threads per line, exchange parts on strided axes) and tile
    // widths one step either side of the heuristic
    for (int ax = 0; ax < 3; ++ax) {
        if (dims[ax] <= 1) continue;
        const bool strided = axis_strided(ax, dims);
        std::vector<const KernelEntry*> ks = kernels_for(dtype, (int)dims[ax]);
        for (const KernelEntry* k : ks) {
            if (k->nparts > 1 && !strided) continue;
            const int l0 = default_logW(k, dtype, strided);
            for (int dl = -1; dl <= 1; ++dl) {
                const int lw = l0 + dl;
                if (lw < 0 || fit_logW(k, lw, dtype) != lw) continue;
                if (k == base.k[ax] && lw == base.logW[ax]) continue;
                PlanChoice c = base;
                c.k[ax] = k;
                c.logW[ax] = lw;
                out.push_back(c);
            }
        }
    }
    // other axis orders with the default kernels
    const int perms[5][3] = {{2, 0, 1}, {1, 2, 0}, {1, 0, 2}, {0, 2, 1}, {0, 1, 2}};
    for (const auto& pm : perms) {
        PlanChoice c = base;
        for (int i = 0; i < 3; ++i) c.order[i] = pm[i];
        out.push_back(c);
    }
    return out;
}

static const char kAxisName[] = "abc";

std::string choice_to_string(const PlanChoice& c, const int64_t dims[3]) {
    std::ostringstream os;
    os << "order=" << kAxisName[c.order[0]] << kAxisName[c.order[1]] << kAxisName[c.order[2]];
    for (int ax = 0; ax < 3; ++ax) {
        os << ";" << kAxisName[ax] << "=";
        if (!c.k[ax] || dims[ax] <= 1) {
            os << "1";
            continue;
        }
        for (int i = 0; i < c.k[ax]->nstages; ++i) os << (i ? "x" : "") << c.k[ax]->radices[i];
        os << "/" << (1 << c.logW[ax]);
        if (c.k[ax]->tpl != default_tpl(c.k[ax])) os << "/" << c.k[ax]->tpl;
        if (c.k[ax]->nparts > 1) os << "/p" << c.k[ax]->nparts;
    }
    return os.str();
}

bool choice_from_string(const char* s, int dtype, const int64_t dims[3], PlanChoice* out, bool check_fit) {
    if (!s) return false;
    PlanChoice c = default_choice(dtype, dims);
    std::string str(s);
    std::stringstream ss(str);
    std::string item;
    bool have_order = false;
    while (std::getline(ss, item, ';')) {
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return false;
        const std::string key = item.substr(0, eq), val = item.substr(eq + 1);
        if (key == "order") {
            if (val.size() != 3) return false;
            bool seen[3] = {false, false, false};
            for (int i = 0; i < 3; ++i) {
                const char* p = strchr(kAxisName, val[i]);
                if (!p || val[i] == 0) return false;
                const int ax = int(p - kAxisName);
                if (seen[ax]) return false;
                seen[ax] = true;
                c.order[i] = ax;
            }
            have_order = true;
        } else if (key.size() == 1 && strchr(kAxisName, key[0]) && key[0]) {
            const int ax = int(strchr(kAxisName, key[0]) - kAxisName);
            if (dims[ax] <= 1) {
                if (val != "1") return false;
                continue;
            }
            const size_t slash = val.find('/');
            if (slash == std::string::npos) return false;
            std::vector<int> rad;
            std::stringstream rs(val.substr(0, slash));
            std::string tok;
            while (std::getline(rs, tok, 'x')) {
                char* end = nullptr;
                const long r = strtol(tok.c_str(), &end, 10);
                if (!end || *end || r < 2) return false;
                rad.push_back((int)r);
            }
            char* end = nullptr;
            const long W = strtol(val.c_str() + slash + 1, &end, 10);
            if (!end || W < 1 || (W & (W - 1))) return false;
            long tpl = 0;   // 0: the sequence's default thread count
            long P = 1;     // parts of each LDS exchange ("/p<P>", strided axes)
            if (*end == '/' && end[1] != 'p') {
                char* end2 = nullptr;
                tpl = strtol(end + 1, &end2, 10);
                if (!end2 || tpl < 1) return false;
                end = end2;
            }
            if (*end == '/' && end[1] == 'p') {
                char* end2 = nullptr;
                P = strtol(end + 2, &end2, 10);
                if (!end2 || (P != 1 && P != 2 && P != 4)) return false;
                end = end2;
            }
            if (*end) return false;
            if (P > 1 && !axis_strided(ax, dims)) return false;
            const KernelEntry* found = nullptr;
            for (const KernelEntry* k : kernels_for(dtype, (int)dims[ax])) {
                if (k->nstages != (int)rad.size()) continue;
                bool eq2 = true;
                for (int i = 0; i < k->nstages; ++i) eq2 = eq2 && k->radices[i] == rad[i];
                if (eq2 && k->tpl == (tpl ? (int)tpl : default_tpl(k)) && k->nparts == (int)P) { found = k; break; }
            }
            if (!found) return false;
            const int lw = ilog2(W);
            if (check_fit && !tile_fits(found, lw, dtype)) return false;
            c.k[ax] = found;
            c.logW[ax] = lw;
        } else {
            return false;
        }
    }
    if (!have_order) return false;
    *out = c;
    return true;
}

int build_passes(const PlanChoice& c, const int64_t dims[3], int64_t batch, PassPlan out[3]) {
    int n = 0;
    for (int i = 0; i < 3; ++i) {
        const int ax = c.order[i];
        if (dims[ax] <= 1) continue;
        PassPlan p;
        p.axis = ax;
        p.L = (int)dims[ax];
        int64_t m1 = batch, m2 = 1;
        for (int j = 0; j < ax; ++j) m1 *= dims[j];
        for (int j = ax + 1; j < 3; ++j) m2 *= dims[j];
        p.M1 = m1;
        p.M2 = m2;
        p.k = c.k[ax];
        p.logW = c.logW[ax];
        p.mode = m2 > 1 ? 1 : 0;
        p.tw = nullptr;
        out[n++] = p;
    }
    return n;
}

hipError_t launch_pass(const PassPlan& p, const void* in, void* out, int conj_in, int conj_out,
                       double scale, hipStream_t s) {
    PassArgs a;
    a.in = in;
    a.out = out;
    a.tw = p.tw;
    a.nlines = p.M1 * p.M2;
    a.M2 = p.M2;
    a.logW = p.logW;
    a.mode = p.mode;
    a.conj_in = conj_in;
    a.conj_out = conj_out;
    a.scale = scale;
    // a kernel with exchanges in parts keeps only part of each line in LDS:
    // strided lines only
    if (p.k->nparts > 1 && p.mode != 1) return hipErrorInvalidValue;
    const int64_t W = int64_t(1) << p.logW;
    const int64_t nblocks = (a.nlines + W - 1) / W;
    const int threads = (int)(W * p.k->tpl);
    const size_t lds = (size_t)tile_lds_elems((int)W, p.L, p.k->nparts) * (p.k->dtype == OFFT_C2C_F64 ? 16 : 8);
    return p.k->launch(a, nblocks, threads, lds, s);
}

}  // namespace offt
