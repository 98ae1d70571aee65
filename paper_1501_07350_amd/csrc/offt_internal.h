// offt_internal.h -- host-side types shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "fft_device.hpp"

namespace offt {

constexpr int kMaxStages = 8;
constexpr int kMaxDims = 5;       // axes of the grids of a D-dimensional plan
constexpr int kTransposeMaxThreads = 512;   // launch bound of every transposing kernel
// Bytes of LDS a pass tile may use: the device's per-workgroup limit (160 KiB
// on gfx950), 64 KiB when no device is visible.
int64_t lds_limit();

using LaunchFn = hipError_t (*)(const PassArgs& a, int64_t nblocks, int threads, size_t lds,
                                hipStream_t s);

// One compiled length-L pass kernel: radix sequence (in stage order), threads
// per line, and its launcher.
struct KernelEntry {
    int dtype;                 // OFFT_C2C_F64 / OFFT_C2C_F32
    int L;
    int nstages;
    int radices[kMaxStages];
    int tpl;                   // threads per line
    int max_threads;           // launch bound the kernel is compiled for
    int nparts;                // parts each LDS exchange runs in (> 1: strided lines only)
    LaunchFn launch;
    LaunchFn launch_t;         // the same tile code as a transposing pass, else nullptr
};

// One kernel case compiled into the persistent batch executor.
struct ManyCase {
    int dtype;
    int L;
    int nstages;
    int radices[kMaxStages];
    int tpl;
};

// A persistent batch executor: its kernel and the cases it dispatches.
struct ManyExecutor {
    const char* name;
    int dtype;
    const ManyCase* cases;
    int ncases;
    const void* kernel;        // work-queue persistent kernel (ManyArgs); null: level kernels only
    const void* level_kernel;  // one tile per workgroup (ManyArgs, int64_t tile_begin)
};

// Registry of all compiled pass kernels (generated tables).
const std::vector<const KernelEntry*>& registry();
// All kernels for (dtype, L), default first.
std::vector<const KernelEntry*> kernels_for(int dtype, int L);

// One axis pass of a plan.
struct PassPlan {
    int axis;                  // 0 = a, 1 = b, 2 = c
    int L;
    int64_t M1, M2;
    int64_t X, Y;              // transposing passes: row map of the other buffer (PassArgs)
    const KernelEntry* k;
    int logW;                  // lines per workgroup = 2^logW
    int mode;                  // 0 contiguous lines, 1 strided lines, 2/3 transposing (PassArgs)
    int xcd = 0;               // tiles in contiguous runs per XCD (PassArgs::xcd_remap)
    int stream = 0;            // streaming loads and stores (PassArgs::stream_io)
    const void* tw;            // device twiddle table for L
    // Slab schedule (PlanChoice::slab): a pass over axis b or c after the
    // whole-grid pass over a runs on `slab` planes (Nb x Nc) at a time, every
    // such pass of one slab before the next slab.  0: the whole grid at once.
    int64_t slab = 0;
    int64_t planes = 0;        // planes the pass covers (batch * Na)
    int64_t plane_elems = 0;   // elements of one plane (Nb * Nc)
    // Column-block schedule (PlanChoice::col): a strided pass over a or b
    // after the whole-grid pass over c runs on blocks of `col` consecutive
    // columns c (out of ncol = Nc), every such pass of one block before the
    // next block.  0: the whole grid at once.
    int64_t col = 0;
    int64_t ncol = 0;
    // a strided pass restricted to one column block (PassArgs): lines per
    // m1 (0: M2), log2 of the block width (-1: none), row length, first column
    int64_t lpm = 0;
    int blk_logw = -1;
    int64_t blk_ld = 0, blk_off = 0;
};

// Pass p restricted to planes [p0, p0 + np) of a slab schedule; *elem_off
// receives the element offset of plane p0.
PassPlan slab_pass(const PassPlan& p, int64_t p0, int64_t np, int64_t* elem_off);
// Pass p restricted to the column block starting at column c0.
PassPlan col_pass(const PassPlan& p, int64_t c0);
// Index of the first pass of a list that runs block by block (slab or column
// schedule), or n.
int slab_start(const PassPlan* ps, int n);

// Grid-data access mode of a pass (plan choices, plan-string suffix):
// kIoAuto streams when the batch of grids exceeds kStreamMinBytes (it then
// cannot stay in the 256 MB Infinity Cache between passes), kIoStream and
// kIoCached force one mode ("/s", "/c").
enum { kIoAuto = 0, kIoStream = 1, kIoCached = 2 };
constexpr int64_t kStreamMinBytes = int64_t(256) << 20;
// Whether a pass over `bytes` of grid data streams under access mode io.
inline int resolve_stream(int io, int64_t bytes) {
    return io == kIoStream || (io == kIoAuto && bytes > kStreamMinBytes) ? 1 : 0;
}

// Plan choice for one grid shape, independent of device memory.
struct PlanChoice {
    int order[3];              // axis order of the passes (axis ids)
    const KernelEntry* k[3];   // per axis id (a, b, c); nullptr for L == 1
    int logW[3];               // per axis id
    int xcd[3] = {0, 0, 0};    // per axis id: XCD-contiguous tile order (plan string "/x")
    int io[3] = {0, 0, 0};     // per axis id: grid-data access mode (kIo*, plan string "/s" or "/c")
    // Output order.  -1: the input's (abc).  0 or 2: reversed (cba), the
    // pass along this axis transposing: axis a reads strided lines of the
    // abc grid and writes cba rows (mode 3), axis c reads abc rows and
    // writes strided lines of the cba grid (mode 2).  Passes before it see
    // the abc grid, passes after it the cba grid.
    int tax = -1;
    // Slab schedule: 0, or the number of planes (Nb x Nc, counted over the
    // batch) per slab.  Requires natural output order (tax < 0) and the pass
    // over a first; the passes over b and c then run slab by slab (plan
    // string ";slab=S"), so that a slab's second pass finds the first pass's
    // output in the Infinity Cache.
    int64_t slab = 0;
    // Column-block schedule: 0, or the number of columns c per block (a power
    // of two dividing Nc).  Requires natural output order and the pass over
    // c first; the passes over b and a then run block by block (plan string
    // ";col=W"), so that a block's second pass finds the first pass's output
    // in the Infinity Cache.  At most one of slab and col is set.
    int64_t col = 0;
};
// Whether a choice's slab or column schedule fits its grid (see
// PlanChoice::slab, PlanChoice::col); with check_tiles, also that every
// blocked pass's tile width divides the block.
bool slab_fits(const PlanChoice& c, const int64_t dims[3]);
bool col_fits(const PlanChoice& c, const int64_t dims[3], bool check_tiles);

// Where an axis pass of a choice runs: on the input's (abc) grid, on the
// reversed (cba) grid, or as the transposing pass between them.
enum AxisGeom { kGeomNatural = 0, kGeomReversed = 1, kGeomTranspose = 2 };
int axis_geom(const PlanChoice& c, int ax);
// The pass of axis ax in geometry g (k and logW filled in, tw left null).
PassPlan make_pass(const int64_t dims[3], int64_t batch, int ax, int g, const KernelEntry* k, int logW,
                   int xcd = 0, int io = kIoAuto);
// Whether the output of a grid has a different memory order in cba than in
// abc (at least two axes longer than 1).
bool reversal_moves_data(const int64_t dims[3]);
// Index of the transposing pass in a pass list, or -1.
int transpose_index(const PassPlan* ps, int n);
// Buffers of pass i: `in` to `out` through the plan's workspace where a
// transposing pass needs one (it never runs in place).  Returns false when
// the workspace is needed and `work` is null.
bool pass_io(const PassPlan* ps, int n, int i, const void* in, void* out, void* work, const void** src,
             void** dst);

// Plan choice for a grid of 4 or 5 axes (every axis on the input's order).
struct NdChoice {
    int ndim = 0;
    int order[kMaxDims];              // axis order of the passes
    const KernelEntry* k[kMaxDims];   // per axis; nullptr for length 1
    int logW[kMaxDims];
    int xcd[kMaxDims] = {0, 0, 0, 0, 0};
    int io[kMaxDims] = {0, 0, 0, 0, 0};
    // slab schedule as PlanChoice::slab: the pass over the first axis first,
    // then every other pass on `slab` blocks (of the product of the other
    // axes) at a time; 0: none
    int64_t slab = 0;
};
bool nd_slab_fits(const NdChoice& c, const int64_t* dims);
PassPlan make_pass_nd(int ndim, const int64_t* dims, int64_t batch, int ax, const KernelEntry* k, int logW,
                      int xcd = 0, int io = kIoAuto);
NdChoice default_choice_nd(int dtype, int ndim, const int64_t* dims);
std::string nd_choice_to_string(const NdChoice& c, const int64_t* dims);
bool nd_choice_from_string(const char* s, int dtype, int ndim, const int64_t* dims, NdChoice* out,
                           bool check_fit = true);
int build_passes_nd(const NdChoice& c, const int64_t* dims, int64_t batch, PassPlan* out);

size_t elem_size(int dtype);
bool smooth235(int64_t n);
std::string choice_to_string(const PlanChoice& c, const int64_t dims[3]);
// Parses a plan string; returns false if it does not parse or does not fit
// dims/dtype (with check_fit, also when a tile exceeds this device's limits).
bool choice_from_string(const char* s, int dtype, const int64_t dims[3], PlanChoice* out, bool check_fit = true);
PlanChoice default_choice(int dtype, const int64_t dims[3]);
// Heuristic plan with the output in reversed (cba) order; equal to
// default_choice when the reversal moves no data.
PlanChoice default_choice_reversed(int dtype, const int64_t dims[3]);
// Candidate plans for tuning (deterministic order, default first).
std::vector<PlanChoice> candidate_choices(int dtype, const int64_t dims[3]);
// The learned selector's candidate list: candidate_choices, then the
// heuristic with one axis's access mode switched (selector.cpp).
std::vector<PlanChoice> selector_candidates(int dtype, const int64_t dims[3], int64_t batch);
// The heuristic pass over `lines` contiguous lines of length L (kernel, tile
// width, access mode for grid data of grid_bytes), twiddles not attached.
PassPlan contiguous_pass(int dtype, int L, int64_t lines, int64_t grid_bytes);
// Pass descriptors (M1, M2, mode, W) for a grid + batch under a choice.
int build_passes(const PlanChoice& c, const int64_t dims[3], int64_t batch, PassPlan out[3]);
// Whether a tile of 2^logW lines of kernel k can be launched: thread limit
// and LDS limit.
bool tile_fits(const KernelEntry* k, int logW, int dtype);
// The same for the kernel's transposing form (false if it has none).
bool tile_fits_transpose(const KernelEntry* k, int logW, int dtype);
// tile_fits or tile_fits_transpose, by geometry.
bool tile_fits_geom(const KernelEntry* k, int logW, int dtype, int g);
// Clamp logW so the tile fits LDS and the thread limit; returns the adjusted value.
int fit_logW(const KernelEntry* k, int logW, int dtype, int g = kGeomNatural);

hipError_t launch_twiddles(void* out, int64_t n, int dtype, hipStream_t s);
// Fills nelem complex elements of `dtype` with values uniform in [-1, 1)
// (tuning data; `key` selects the stream).
hipError_t launch_fill_uniform(void* out, int64_t nelem, int dtype, uint64_t key, hipStream_t s);
hipError_t launch_pass(const PassPlan& p, const void* in, void* out, int conj_in, int conj_out,
                       double scale, hipStream_t s);

void set_error(int code);

}  // namespace offt
