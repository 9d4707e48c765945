// Host-side helpers shared by the s7 translation units: error reporting,
// argument checks, workspace layout and tile choice.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/s7.h"
#include "s7_device.hpp"

namespace s7 {

void set_error(const char* fmt, ...);
void clear_error();

#define S7_HIP(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::s7::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                            __LINE__);                                                    \
            return S7_EHIP;                                                               \
        }                                                                                 \
    } while (0)

#define S7_CHECK_LAUNCH() S7_HIP(hipGetLastError())

// Largest mesh: cell indices are 32-bit, and a thread index or a grid-stride
// loop may run up to 2^20 past the last cell, so N stays 2^21 below 2^31.
constexpr long long kMaxCells = (1ll << 31) - (1ll << 21);
inline bool dims_ok(s7_dims d) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return false;
    long long n = (long long)d.nx * d.ny * d.nz;
    return n <= kMaxCells;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

inline size_t elt_size(int prec) { return prec == S7_FP32 ? 4 : 2; }

inline int cell_blocks_for(long long n) { return (int)((n + kThreads - 1) / kThreads); }

// Workgroups of the streaming passes: at most 256 by default, at least one per
// 2048 cells.  The grid strides over the arrays in tiles of kThreads vector
// accesses, so all workgroups sweep the same region of each array together;
// with 256 workgroups (one per CU) these mixed read/write streams reached the
// highest HBM rate.
inline int stream_blocks_for(long long n, int cap) {
    long long b = (n + kThreads * 8 - 1) / (kThreads * 8);
    if (b < 1) b = 1;
    if (cap <= 0) cap = 256;
    if (cap > kSingleMax) cap = kSingleMax;  // the streaming passes always finish in-kernel
    if (b > cap) b = cap;
    return (int)b;
}

// Workspace of one system: [State][partials][group partials][counter]
// [batch control][coef copies][6 vectors of T: r, r0, p, s, y, q][d: FP32].
struct Layout {
    size_t off_state, off_part, off_gpart, off_cnt, off_ctl, off_coef, off_vec, off_d, bytes;
    int ncoef;
    int cell_blocks, stream_blocks, groups;
    size_t elt;
    size_t n;
};

// ncoef: working coefficient copies (0: 6 with Jacobi scaling, else 7, the
// 7-point operator).
Layout make_layout(s7_dims d, int prec, const s7_options& o, int ncoef = 0);

void options_or_default(const s7_options* in, s7_options& out);

// ---------------------------------------------------------------- autotuning cache
// Tuned launch parameters per size class.  kind: TUNE_SINGLE (val: schedule,
// stream_blocks) or TUNE_BATCH (val: chunk_cells, persistent grid).  Classes
// are half-octaves of the cell count (and, for batches, of the system count).
enum TuneKind { TUNE_SINGLE = 1, TUNE_BATCH = 2, TUNE_BATCH9 = 3 };
struct TuneKey {
    int kind, tag, unit, nbucket, sbucket;
    bool operator<(const TuneKey& o) const;
};
inline int size_bucket(double v) { return v < 1.0 ? 0 : (int)floor(2.0 * log2(v)); }
bool tune_lookup(const TuneKey& k, int (&val)[4]);
void tune_store(const TuneKey& k, const int (&val)[4]);
// Appends one line to the file named by S7_TUNE_LOG, if set (the timing of
// each autotuning trial).
void tune_log(const char* line);

// ---------------------------------------------------------------- batch engine
// Runs many systems together: the batched entry point and the request queue
// both drive it.  Each system brings its own workspace slice (s7_workspace_bytes
// of its dims and precision).  The engine's tables (one BSys per resident
// system and the launch-global words) live in a separate device region of
// engine_table_bytes(capacity).
struct EngineJob {
    s7_dims d;            // nz = 1 for the 2D 9-point operator
    const float* coef[7];
    const float* coef9[2];  // the 2D 9-point operator's coefficients 7 and 8 (nw, ne)
    const double* b;
    double* x;
    double rtol;
    int32_t max_iter;
    int32_t prec;
    char* ws;         // the job's workspace slice
    size_t ws_bytes;
    s7_info info;     // filled when the job is finished
    int finished;     // 1 once info is final
    void* user;       // owner's handle
    int op = 0;       // 0: 3D 7-point, 1: 2D 9-point
    // engine-private
    int stage, tag;
    Layout lo;
    double t_start_ms;
};

size_t engine_table_bytes(int capacity);

struct BSys;  // one system of a persistent launch (device table entry)

class BatchEngine {
  public:
    // use_graph: replay the persistent launch from a captured hipGraph, for
    // callers whose resident set repeats (the batched entry point).  Jobs of
    // both operators (EngineJob::op) may be resident together: one persistent
    // launch runs them all.
    BatchEngine(char* tables, int capacity, const s7_options& o, hipStream_t stream,
                bool use_graph = false);
    ~BatchEngine();
    BatchEngine(const BatchEngine&) = delete;
    BatchEngine& operator=(const BatchEngine&) = delete;
    // Takes part from the next step on; the job's arrays must stay valid until finished.
    int add(EngineJob* job);
    // Advances every resident job: starts new ones, then runs one persistent launch
    // in which each job continues its solve (iterations, refinement steps and
    // epilogue all run on the device).  In the launch each job runs at most
    // `epoch_iters` BiCGStab iterations; with epoch_iters <= 0 every job runs until
    // `slice_ms` of device wall-clock time have passed, then parks at its next phase
    // boundary, so one launch takes about slice_ms whatever the sizes.  Finished jobs
    // leave the resident set with their info filled.  Returns S7_OK or an error.
    int step(int epoch_iters, double slice_ms = 2.0);
    int resident() const { return (int)jobs_.size(); }
    // Picks chunk_cells and the persistent grid for the size class of the resident
    // jobs (all not yet started), by timing short trials on synthetic contents of
    // their workspaces, unless the class is cached.  Call before the first step.
    int tune();

  private:
    int read_states(std::vector<State>& h);
    // Uploads `table` and runs one persistent launch (arm + kernel), then waits for it.
    int launch(const std::vector<BSys>& table, int epoch_key, int chunk, int grid, long long slice = 0);
    char* tables_;
    int cap_;
    s7_options o_;
    hipStream_t st_;
    bool graph_;
    int chunk_;     // cells per work item of the persistent kernel
    int grid_cap_;  // most workgroups of a persistent launch
    double ticks_per_ms_ = 100000.0;  // device wall clock
    State* host_states_ = nullptr;  // pinned, cap_ entries
    std::vector<EngineJob*> jobs_;
};

}  // namespace s7
