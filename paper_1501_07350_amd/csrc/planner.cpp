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

bool tile_fits_transpose(const KernelEntry* k, int logW, int dtype) {
    if (!k || !k->launch_t || logW < 0) return false;
    const int64_t W = int64_t(1) << logW;
    if (W * k->tpl > kTransposeMaxThreads) return false;
    return tile_lds_elems_transpose((int)W, k->L, k->nparts) * (int64_t)elem_size(dtype) <= lds_limit();
}

bool tile_fits_geom(const KernelEntry* k, int logW, int dtype, int g) {
    return g == kGeomTranspose ? tile_fits_transpose(k, logW, dtype) : tile_fits(k, logW, dtype);
}

int fit_logW(const KernelEntry* k, int logW, int dtype, int g) {
    if (!k) return 0;
    while (logW > 0 && !tile_fits_geom(k, logW, dtype, g)) --logW;
    return logW;
}

// ---- geometry of the passes ---------------------------------------------------

int axis_geom(const PlanChoice& c, int ax) {
    if (c.tax < 0) return kGeomNatural;
    if (ax == c.tax) return kGeomTranspose;
    int pa = 0, pt = 0;
    for (int i = 0; i < 3; ++i) {
        if (c.order[i] == ax) pa = i;
        if (c.order[i] == c.tax) pt = i;
    }
    return pa < pt ? kGeomNatural : kGeomReversed;
}

// On the abc grid the lines of axis ax form the [M1][L][M2] view with M1 the
// product of the axes before it (times the batch) and M2 of those after it;
// on the cba grid the two swap.  The transposing pass keeps the strided view
// of its strided side: the abc grid for axis a (rows written to the cba
// grid), the cba grid for axis c (rows read from the abc grid).  In both the
// row of line m1*M2 + m2 is m1*M2 + (m2 mod X)*Y + m2 div X with X the
// length of the opposite end axis and Y = Nb.
PassPlan make_pass(const int64_t dims[3], int64_t batch, int ax, int g, const KernelEntry* k, int logW, int xcd,
                   int io) {
    PassPlan p;
    p.axis = ax;
    p.L = (int)dims[ax];
    p.k = k;
    p.logW = logW;
    p.xcd = xcd;
    p.stream = k ? resolve_stream(io, dims[0] * dims[1] * dims[2] * batch * (int64_t)elem_size(k->dtype)) : 0;
    p.tw = nullptr;
    p.X = 1;
    p.Y = 1;
    int64_t before = 1, after = 1;
    for (int j = 0; j < ax; ++j) before *= dims[j];
    for (int j = ax + 1; j < 3; ++j) after *= dims[j];
    if (g == kGeomTranspose) {
        p.M1 = batch;
        p.M2 = before * after;
        p.X = dims[2 - ax];
        p.Y = dims[1];
        p.mode = ax == 0 ? 3 : 2;
    } else if (g == kGeomReversed) {
        p.M1 = batch * after;
        p.M2 = before;
        p.mode = before > 1 ? 1 : 0;
    } else {
        p.M1 = batch * before;
        p.M2 = after;
        p.mode = after > 1 ? 1 : 0;
    }
    return p;
}

bool reversal_moves_data(const int64_t dims[3]) {
    int n = 0;
    for (int ax = 0; ax < 3; ++ax) n += dims[ax] > 1;
    return n >= 2;
}

int transpose_index(const PassPlan* ps, int n) {
    for (int i = 0; i < n; ++i)
        if (ps[i].mode >= 2) return i;
    return -1;
}

// Without a transposing pass (or with one first and distinct buffers) pass 0
// reads `in` and every pass writes `out`.  Passes before a later transposing
// pass run in the workspace, which it then reads; a transposing first pass
// with in == out writes the workspace and the second pass brings the data
// back to `out`.
bool pass_io(const PassPlan* ps, int n, int i, const void* in, void* out, void* work, const void** src,
             void** dst) {
    const int tp = transpose_index(ps, n);
    if (tp < 0 || (tp == 0 && in != out)) {
        *src = i == 0 ? in : out;
        *dst = out;
        return true;
    }
    if (!work) return false;
    if (tp == 0) {
        *src = i == 0 ? in : (i == 1 ? (const void*)work : (const void*)out);
        *dst = i == 0 ? work : out;
        return true;
    }
    if (i < tp) {
        *src = i == 0 ? in : (const void*)work;
        *dst = work;
    } else {
        *src = i == tp ? (const void*)work : (const void*)out;
        *dst = out;
    }
    return true;
}

static int max_radix(const KernelEntry* k) {
    int maxr = 0;
    for (int i = 0; i < k->nstages; ++i) maxr = std::max(maxr, k->radices[i]);
    return maxr;
}

// Heuristic tile width: strided lines get 256-byte row segments (16 columns
// of complex128, 32 of complex64), and radix-32 kernels 32 columns in both
// precisions; contiguous lines ~512 threads per workgroup for complex128 and
// ~256 for complex64.
static int strided_logW(const KernelEntry* k, int dtype) {
    return max_radix(k) >= 32 ? 5 : (dtype == OFFT_C2C_F64 ? 4 : 5);
}

static int default_logW(const KernelEntry* k, int dtype, bool strided) {
    if (!k) return 0;
    int logW;
    if (strided)
        logW = strided_logW(k, dtype);
    else
        logW = ilog2(std::max<int64_t>(1, (dtype == OFFT_C2C_F64 ? 512 : 256) / k->tpl));
    return fit_logW(k, logW, dtype);
}

// Default kernel of an axis: the first in kernels_for() order whose tile at the
// heuristic width fits; contiguous axes take the first kernel with whole-line
// exchanges and radix <= 16, complex64 ones first looking for radix <= 8 at
// the default threads per line (over the 2200 grids of the selector's data
// set, such a kernel at the same width made the complex64 transform faster in
// 84% of the grids where the radix-16 kernel was the default, geometric mean
// 0.93 of the time, 0.92 for axes up to 128 points).  Strided axes of length >= 512 look first at
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
    if (!strided && dtype == OFFT_C2C_F32)
        for (const KernelEntry* k : kernels_for(dtype, L))
            if (k->nparts == 1 && max_radix(k) <= 8 && k->tpl * max_radix(k) == L) ks.push_back(k);
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

// Default tile order: XCD-contiguous for strided lines.  Over the 2200 grids
// of the selector's data set (axes 16..1024, MI355X) that order made strided
// passes faster in 59-75% of the grids above 64 MiB (geometric mean 0.93 of
// the time) and slightly faster below; on contiguous lines it was neutral to
// slower, and transposing passes keep the launch order.  With streaming
// accesses (grids above the Infinity Cache) the launch order was faster for
// lines strided by 2 MiB or more: 6% for pass a at 1024^3 complex64, 3% at
// 512^3 complex64.
constexpr int64_t kLongStrideBytes = int64_t(2) << 20;
static int default_xcd(int g, bool strided, bool streamed_long_stride = false) {
    return g != kGeomTranspose && strided && !streamed_long_stride ? 1 : 0;
}
// Whether the heuristic's pass along `ax` (natural geometry, one grid) streams
// over lines strided by kLongStrideBytes or more.
static bool streamed_long_stride(int dtype, const int64_t* dims, int ndim, int ax) {
    int64_t n = 1, after = 1;
    for (int j = 0; j < ndim; ++j) n *= dims[j];
    for (int j = ax + 1; j < ndim; ++j) after *= dims[j];
    const int64_t es = (int64_t)elem_size(dtype);
    return resolve_stream(kIoAuto, n * es) && after * es >= kLongStrideBytes;
}

// Default kernel of a transposing pass: for L >= 512 the first radix <= 16
// kernel whose exchanges and row side run in 2 parts (half the LDS of a
// whole-line tile, so two workgroups share a CU: on MI355X at 512^3 these
// ran the transposing pass 13-17% faster than whole-line tiles), else the
// first whole-line kernel with radix <= 16.  Tiles of 16 lines.
static const KernelEntry* default_kernel_transpose(int dtype, int L) {
    if (L >= 512)
        for (const KernelEntry* k : kernels_for(dtype, L))
            if (k->nparts == 2 && k->launch_t && max_radix(k) <= 16 && tile_fits_transpose(k, 4, dtype)) return k;
    for (const KernelEntry* k : kernels_for(dtype, L))
        if (k->nparts == 1 && k->launch_t && max_radix(k) <= 16) return k;
    for (const KernelEntry* k : kernels_for(dtype, L))
        if (k->nparts == 1 && k->launch_t) return k;
    return nullptr;
}

// The heuristic kernel and width of every axis, for the geometry the
// choice's order and output order give it.
static void assign_default_kernels(PlanChoice& c, int dtype, const int64_t dims[3]) {
    for (int ax = 0; ax < 3; ++ax) {
        c.k[ax] = nullptr;
        c.logW[ax] = 0;
        if (dims[ax] <= 1) continue;
        const int g = axis_geom(c, ax);
        const KernelEntry* k;
        int logW;
        if (g == kGeomTranspose) {
            k = default_kernel_transpose(dtype, (int)dims[ax]);
            logW = k ? fit_logW(k, 4, dtype, g) : 0;
        } else {
            const bool strided = make_pass(dims, 1, ax, g, nullptr, 0).M2 > 1;
            k = default_kernel(dtype, (int)dims[ax], strided);
            logW = default_logW(k, dtype, strided);
        }
        if (k) {
            c.k[ax] = k;
            c.logW[ax] = logW;
            c.xcd[ax] = default_xcd(g, make_pass(dims, 1, ax, g, nullptr, 0).M2 > 1,
                                    g == kGeomNatural && streamed_long_stride(dtype, dims, 3, ax));
        }
    }
}

PassPlan contiguous_pass(int dtype, int L, int64_t lines, int64_t grid_bytes) {
    PassPlan p;
    p.axis = 2;
    p.L = L;
    p.M1 = lines;
    p.M2 = 1;
    p.X = 1;
    p.Y = 1;
    p.mode = 0;
    p.xcd = 0;
    p.tw = nullptr;
    p.k = default_kernel(dtype, L, false);
    p.logW = default_logW(p.k, dtype, false);
    p.stream = resolve_stream(kIoAuto, grid_bytes);
    return p;
}

PlanChoice default_choice(int dtype, const int64_t dims[3]) {
    PlanChoice c;
    c.order[0] = 2; c.order[1] = 1; c.order[2] = 0;   // c, then b, then a
    c.tax = -1;
    assign_default_kernels(c, dtype, dims);
    return c;
}

// Reversed output: passes c, b, a with the pass along a transposing (strided
// abc lines in, cba rows out), so the first pass reads contiguous lines and
// only pass b runs on strided lines of one buffer; without an axis a, the
// pass along c transposes (abc rows in, strided cba lines out).
PlanChoice default_choice_reversed(int dtype, const int64_t dims[3]) {
    if (!reversal_moves_data(dims)) return default_choice(dtype, dims);
    PlanChoice c;
    c.order[0] = 2; c.order[1] = 1; c.order[2] = 0;
    c.tax = dims[0] > 1 ? 0 : 2;
    assign_default_kernels(c, dtype, dims);
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
    // the heuristic with one axis's tile order switched (launch order <->
    // XCD-contiguous)
    for (int ax = 0; ax < 3; ++ax) {
        if (dims[ax] <= 1 || !base.k[ax]) continue;
        PlanChoice c = base;
        c.xcd[ax] = !base.xcd[ax];
        out.push_back(c);
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

static const char kAxisName[] = "abcde";

// ---- plan strings ---------------------------------------------------------------
// One axis: "<radix sequence>/<tile width>[/<threads per line>][/p<parts>][/x][/s|/c]",
// or "1" for a length-1 axis ("/x": XCD-contiguous tile order; "/s", "/c":
// streaming or cached grid-data accesses, by default chosen from the grid's
// size).

static void axis_to_string(std::ostringstream& os, const KernelEntry* k, int logW, int64_t len, int xcd, int io) {
    if (!k || len <= 1) {
        os << "1";
        return;
    }
    for (int i = 0; i < k->nstages; ++i) os << (i ? "x" : "") << k->radices[i];
    os << "/" << (1 << logW);
    if (k->tpl != default_tpl(k)) os << "/" << k->tpl;
    if (k->nparts > 1) os << "/p" << k->nparts;
    if (xcd) os << "/x";
    if (io == kIoStream) os << "/s";
    if (io == kIoCached) os << "/c";
}

namespace {
struct AxisSpec {
    bool given = false;
    std::vector<int> rad;
    long W = 0, tpl = 0, P = 1;
    int xcd = 0;
    int io = kIoAuto;
};
}  // namespace

static bool parse_axis_spec(const std::string& val, AxisSpec* sp) {
    sp->given = true;
    const size_t slash = val.find('/');
    if (slash == std::string::npos) return false;
    std::stringstream rs(val.substr(0, slash));
    std::string tok;
    while (std::getline(rs, tok, 'x')) {
        char* end = nullptr;
        const long r = strtol(tok.c_str(), &end, 10);
        if (!end || *end || r < 2) return false;
        sp->rad.push_back((int)r);
    }
    char* end = nullptr;
    sp->W = strtol(val.c_str() + slash + 1, &end, 10);
    if (!end || sp->W < 1 || (sp->W & (sp->W - 1))) return false;
    if (*end == '/' && end[1] >= '0' && end[1] <= '9') {   // threads per line (default: the sequence's)
        char* end2 = nullptr;
        sp->tpl = strtol(end + 1, &end2, 10);
        if (!end2 || sp->tpl < 1) return false;
        end = end2;
    }
    if (*end == '/' && end[1] == 'p') {   // parts of each LDS exchange (strided axes)
        char* end2 = nullptr;
        sp->P = strtol(end + 2, &end2, 10);
        if (!end2 || (sp->P != 1 && sp->P != 2 && sp->P != 4)) return false;
        end = end2;
    }
    if (end[0] == '/' && end[1] == 'x' && (end[2] == 0 || end[2] == '/')) {   // XCD-contiguous tile order
        sp->xcd = 1;
        end += 2;
    }
    if (end[0] == '/' && (end[1] == 's' || end[1] == 'c') && end[2] == 0) {   // grid-data access mode
        sp->io = end[1] == 's' ? kIoStream : kIoCached;
        end += 2;
    }
    return *end == 0;
}

static const KernelEntry* find_kernel(int dtype, int L, const AxisSpec& sp) {
    for (const KernelEntry* k : kernels_for(dtype, L)) {
        if (k->nstages != (int)sp.rad.size()) continue;
        bool eq = true;
        for (int i = 0; i < k->nstages; ++i) eq = eq && k->radices[i] == sp.rad[i];
        if (eq && k->tpl == (sp.tpl ? (int)sp.tpl : default_tpl(k)) && k->nparts == (int)sp.P) return k;
    }
    return nullptr;
}

// "order=<axis letters>": a permutation of the first ndim letters
static bool parse_order(const std::string& val, int ndim, int* order) {
    if ((int)val.size() != ndim) return false;
    bool seen[kMaxDims] = {false, false, false, false, false};
    for (int i = 0; i < ndim; ++i) {
        const char* p = val[i] ? strchr(kAxisName, val[i]) : nullptr;
        if (!p || p - kAxisName >= ndim) return false;
        const int ax = int(p - kAxisName);
        if (seen[ax]) return false;
        seen[ax] = true;
        order[i] = ax;
    }
    return true;
}

std::string choice_to_string(const PlanChoice& c, const int64_t dims[3]) {
    std::ostringstream os;
    os << "order=" << kAxisName[c.order[0]] << kAxisName[c.order[1]] << kAxisName[c.order[2]];
    if (c.tax >= 0) os << ";rev=" << kAxisName[c.tax];
    for (int ax = 0; ax < 3; ++ax) {
        os << ";" << kAxisName[ax] << "=";
        axis_to_string(os, c.k[ax], c.logW[ax], dims[ax], c.xcd[ax], c.io[ax]);
    }
    if (c.slab > 0) os << ";slab=" << c.slab;
    if (c.col > 0) os << ";col=" << c.col;
    return os.str();
}

bool slab_fits(const PlanChoice& c, const int64_t dims[3]) {
    return c.slab == 0 || (c.slab > 0 && c.col == 0 && c.tax < 0 && c.order[0] == 0 && dims[0] > 1 &&
                           dims[1] * dims[2] > 1);
}

bool col_fits(const PlanChoice& c, const int64_t dims[3], bool check_tiles) {
    if (c.col == 0) return true;
    const int64_t w = c.col;
    if (w < 1 || (w & (w - 1)) || c.slab != 0 || c.tax >= 0 || c.order[0] != 2 || dims[2] <= 1 ||
        dims[0] * dims[1] <= 1 || dims[2] % w != 0 || w >= dims[2])
        return false;
    // every blocked pass takes whole tiles of one block row: W lines of one
    // m1 are W consecutive columns
    if (check_tiles)
        for (int ax = 0; ax < 2; ++ax)
            if (dims[ax] > 1 && (!c.k[ax] || (int64_t(1) << c.logW[ax]) > w)) return false;
    return true;
}

// Planes per slab from a plan string: a decimal count of 1 to 2^40.
static bool parse_slab(const std::string& val, int64_t* out) {
    if (val.empty() || val.size() > 13) return false;
    int64_t v = 0;
    for (char ch : val) {
        if (ch < '0' || ch > '9') return false;
        v = v * 10 + (ch - '0');
    }
    if (v < 1 || v > (int64_t(1) << 40)) return false;
    *out = v;
    return true;
}

PassPlan slab_pass(const PassPlan& p, int64_t p0, int64_t np, int64_t* elem_off) {
    PassPlan q = p;
    q.M1 = p.M1 / p.planes * np;
    *elem_off = p0 * p.plane_elems;
    return q;
}

PassPlan col_pass(const PassPlan& p, int64_t c0) {
    PassPlan q = p;
    int lw = 0;
    while ((int64_t(1) << lw) < p.col) ++lw;
    q.blk_logw = lw;
    q.blk_ld = p.ncol;
    q.blk_off = c0;
    q.lpm = p.M2 / p.ncol * p.col;   // rows of the m1 (M2 / Nc of them) times the block's columns
    return q;
}

int slab_start(const PassPlan* ps, int n) {
    for (int i = 0; i < n; ++i)
        if (ps[i].slab > 0 || ps[i].col > 0) return i;
    return n;
}

bool choice_from_string(const char* s, int dtype, const int64_t dims[3], PlanChoice* out, bool check_fit) {
    if (!s) return false;
    AxisSpec spec[3];
    PlanChoice c;
    c.tax = -1;
    std::string str(s);
    std::stringstream ss(str);
    std::string item;
    bool have_order = false;
    while (std::getline(ss, item, ';')) {
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return false;
        const std::string key = item.substr(0, eq), val = item.substr(eq + 1);
        if (key == "order") {
            if (!parse_order(val, 3, c.order)) return false;
            have_order = true;
        } else if (key == "rev") {
            if (val == "a") c.tax = 0;
            else if (val == "c") c.tax = 2;
            else return false;
        } else if (key == "slab") {
            if (!parse_slab(val, &c.slab)) return false;
        } else if (key == "col") {
            if (!parse_slab(val, &c.col)) return false;
        } else if (key.size() == 1 && key[0] >= 'a' && key[0] <= 'c') {
            const int ax = key[0] - 'a';
            if (dims[ax] <= 1) {
                if (val != "1") return false;
                continue;
            }
            if (!parse_axis_spec(val, &spec[ax])) return false;
        } else {
            return false;
        }
    }
    if (!have_order) return false;
    if (c.tax >= 0 && (!reversal_moves_data(dims) || dims[c.tax] <= 1)) return false;
    if (!slab_fits(c, dims) || !col_fits(c, dims, false)) return false;
    // axes the string leaves out take the heuristic's kernel for their geometry
    assign_default_kernels(c, dtype, dims);
    for (int ax = 0; ax < 3; ++ax) {
        if (!spec[ax].given) continue;
        const AxisSpec& sp = spec[ax];
        const int g = axis_geom(c, ax);
        const bool strided = g == kGeomTranspose || make_pass(dims, 1, ax, g, nullptr, 0).M2 > 1;
        if (sp.P > 1 && !strided) return false;
        const KernelEntry* found = find_kernel(dtype, (int)dims[ax], sp);
        if (!found || (g == kGeomTranspose && !found->launch_t)) return false;
        const int lw = ilog2(sp.W);
        if (check_fit && !tile_fits_geom(found, lw, dtype, g)) return false;
        c.k[ax] = found;
        c.logW[ax] = lw;
        c.xcd[ax] = sp.xcd;
        c.io[ax] = sp.io;
    }
    if (!col_fits(c, dims, true)) return false;
    *out = c;
    return true;
}

// ---- grids of more than three dimensions -------------------------------------

PassPlan make_pass_nd(int ndim, const int64_t* dims, int64_t batch, int ax, const KernelEntry* k, int logW,
                      int xcd, int io) {
    PassPlan p;
    p.axis = ax;
    p.L = (int)dims[ax];
    p.k = k;
    p.logW = logW;
    p.xcd = xcd;
    int64_t bytes = batch;
    for (int j = 0; j < ndim; ++j) bytes *= dims[j];
    p.stream = k ? resolve_stream(io, bytes * (int64_t)elem_size(k->dtype)) : 0;
    p.tw = nullptr;
    p.X = 1;
    p.Y = 1;
    int64_t before = 1, after = 1;
    for (int j = 0; j < ax; ++j) before *= dims[j];
    for (int j = ax + 1; j < ndim; ++j) after *= dims[j];
    p.M1 = batch * before;
    p.M2 = after;
    p.mode = after > 1 ? 1 : 0;
    return p;
}

// Heuristic: passes from the last (contiguous) axis to the first, each axis
// with the kernel and width the three-dimensional heuristic gives a line of
// its length and stride kind.
NdChoice default_choice_nd(int dtype, int ndim, const int64_t* dims) {
    NdChoice c;
    c.ndim = ndim;
    for (int i = 0; i < ndim; ++i) c.order[i] = ndim - 1 - i;
    for (int ax = 0; ax < ndim; ++ax) {
        c.k[ax] = nullptr;
        c.logW[ax] = 0;
        if (dims[ax] <= 1) continue;
        const bool strided = make_pass_nd(ndim, dims, 1, ax, nullptr, 0).M2 > 1;
        const KernelEntry* k = default_kernel(dtype, (int)dims[ax], strided);
        if (k) {
            c.k[ax] = k;
            c.logW[ax] = default_logW(k, dtype, strided);
            c.xcd[ax] = default_xcd(kGeomNatural, strided, streamed_long_stride(dtype, dims, ndim, ax));
        }
    }
    return c;
}

std::string nd_choice_to_string(const NdChoice& c, const int64_t* dims) {
    std::ostringstream os;
    os << "order=";
    for (int i = 0; i < c.ndim; ++i) os << kAxisName[c.order[i]];
    for (int ax = 0; ax < c.ndim; ++ax) {
        os << ";" << kAxisName[ax] << "=";
        axis_to_string(os, c.k[ax], c.logW[ax], dims[ax], c.xcd[ax], c.io[ax]);
    }
    if (c.slab > 0) os << ";slab=" << c.slab;
    return os.str();
}

bool nd_slab_fits(const NdChoice& c, const int64_t* dims) {
    int64_t rest = 1;
    for (int ax = 1; ax < c.ndim; ++ax) rest *= dims[ax];
    return c.slab == 0 || (c.slab > 0 && c.ndim >= 2 && c.order[0] == 0 && dims[0] > 1 && rest > 1);
}

bool nd_choice_from_string(const char* s, int dtype, int ndim, const int64_t* dims, NdChoice* out,
                           bool check_fit) {
    if (!s || ndim < 1 || ndim > kMaxDims) return false;
    AxisSpec spec[kMaxDims];
    NdChoice c = default_choice_nd(dtype, ndim, dims);
    std::string str(s);
    std::stringstream ss(str);
    std::string item;
    bool have_order = false;
    while (std::getline(ss, item, ';')) {
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return false;
        const std::string key = item.substr(0, eq), val = item.substr(eq + 1);
        if (key == "order") {
            if (!parse_order(val, ndim, c.order)) return false;
            have_order = true;
        } else if (key == "slab") {
            if (!parse_slab(val, &c.slab)) return false;
        } else if (key.size() == 1 && key[0] >= 'a' && key[0] < 'a' + ndim) {
            const int ax = key[0] - 'a';
            if (dims[ax] <= 1) {
                if (val != "1") return false;
                continue;
            }
            if (!parse_axis_spec(val, &spec[ax])) return false;
        } else {
            return false;
        }
    }
    if (!have_order || !nd_slab_fits(c, dims)) return false;
    for (int ax = 0; ax < ndim; ++ax) {
        if (!spec[ax].given) continue;
        const bool strided = make_pass_nd(ndim, dims, 1, ax, nullptr, 0).M2 > 1;
        if (spec[ax].P > 1 && !strided) return false;
        const KernelEntry* found = find_kernel(dtype, (int)dims[ax], spec[ax]);
        if (!found) return false;
        const int lw = ilog2(spec[ax].W);
        if (check_fit && !tile_fits(found, lw, dtype)) return false;
        c.k[ax] = found;
        c.logW[ax] = lw;
        c.xcd[ax] = spec[ax].xcd;
        c.io[ax] = spec[ax].io;
    }
    *out = c;
    return true;
}

static int64_t grid_elems_nd(int ndim, const int64_t* dims) {
    int64_t n = 1;
    for (int i = 0; i < ndim; ++i) n *= dims[i];
    return n;
}

// Every pass after the first on slabs of `slab` planes (blocks of
// plane_elems elements, `planes` of them); access modes resolved for one
// slab's bytes (it may stay cached between the passes).
static void set_slab(PassPlan* out, int n, int64_t planes, int64_t plane_elems, int64_t slab_planes, const int* io) {
    const int64_t slab = std::min(slab_planes, planes);
    for (int i = 1; i < n; ++i) {
        out[i].slab = slab;
        out[i].planes = planes;
        out[i].plane_elems = plane_elems;
        if (out[i].k)
            out[i].stream = resolve_stream(io[out[i].axis], slab * plane_elems * (int64_t)elem_size(out[i].k->dtype));
    }
}

int build_passes_nd(const NdChoice& c, const int64_t* dims, int64_t batch, PassPlan* out) {
    int n = 0;
    for (int i = 0; i < c.ndim; ++i) {
        const int ax = c.order[i];
        if (dims[ax] <= 1) continue;
        out[n++] = make_pass_nd(c.ndim, dims, batch, ax, c.k[ax], c.logW[ax], c.xcd[ax], c.io[ax]);
    }
    if (c.slab > 0 && nd_slab_fits(c, dims))
        set_slab(out, n, batch * dims[0], dims[0] > 0 ? grid_elems_nd(c.ndim, dims) / dims[0] : 0, c.slab, c.io);
    return n;
}

int build_passes(const PlanChoice& c, const int64_t dims[3], int64_t batch, PassPlan out[3]) {
    int n = 0;
    for (int i = 0; i < 3; ++i) {
        const int ax = c.order[i];
        if (dims[ax] <= 1) continue;
        out[n++] = make_pass(dims, batch, ax, axis_geom(c, ax), c.k[ax], c.logW[ax], c.xcd[ax], c.io[ax]);
    }
    if (c.slab > 0 && slab_fits(c, dims)) set_slab(out, n, batch * dims[0], dims[1] * dims[2], c.slab, c.io);
    if (c.col > 0 && col_fits(c, dims, true)) {
        // every pass after the one over c, on blocks of columns; access modes
        // resolved for one block's bytes
        for (int i = 1; i < n; ++i) {
            out[i].col = c.col;
            out[i].ncol = dims[2];
            if (out[i].k)
                out[i].stream = resolve_stream(c.io[out[i].axis], batch * dims[0] * dims[1] * c.col *
                                                                      (int64_t)elem_size(out[i].k->dtype));
        }
    }
    return n;
}

hipError_t launch_pass(const PassPlan& p, const void* in, void* out, int conj_in, int conj_out,
                       double scale, hipStream_t s) {
    PassArgs a;
    a.in = in;
    a.out = out;
    a.tw = p.tw;
    a.lpm = p.lpm > 0 ? p.lpm : p.M2;
    a.nlines = p.M1 * a.lpm;
    a.M2 = p.M2;
    a.blk_logw = p.blk_logw;
    a.blk_ld = p.blk_ld;
    a.blk_off = p.blk_off;
    a.X = p.X;
    a.Y = p.Y;
    a.logW = p.logW;
    a.mode = p.mode;
    a.xcd_remap = p.xcd;
    a.stream_io = p.stream;
    a.conj_in = conj_in;
    a.conj_out = conj_out;
    a.scale = scale;
    // a kernel with exchanges in parts keeps only part of each line in LDS:
    // strided lines (or the strided side of a transposing pass) only
    if (p.k->nparts > 1 && p.mode == 0) return hipErrorInvalidValue;
    const int64_t W = int64_t(1) << p.logW;
    const int64_t nblocks = (a.nlines + W - 1) / W;
    const int threads = (int)(W * p.k->tpl);
    if (p.mode >= 2) {
        // transposing pass: never in place (its row side and strided side
        // cover the same elements in different orders)
        if (!p.k->launch_t || in == out || p.X < 1 || p.Y < 1 || p.X * p.Y != p.M2) return hipErrorInvalidValue;
        const size_t lds_t = (size_t)tile_lds_elems_transpose((int)W, p.L, p.k->nparts) * elem_size(p.k->dtype);
        return p.k->launch_t(a, nblocks, threads, lds_t, s);
    }
    const size_t lds = (size_t)tile_lds_elems((int)W, p.L, p.k->nparts) * (p.k->dtype == OFFT_C2C_F64 ? 16 : 8);
    return p.k->launch(a, nblocks, threads, lds, s);
}

}  // namespace offt
