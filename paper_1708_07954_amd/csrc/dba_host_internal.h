// dba_host_internal.h -- the handle and helpers shared by the host
// translation units of libdba.so.
#pragma once
#include "dba.h"
#include "dba_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace dba {
namespace host {

using dba::Ctrl;
using dba::DevArrays;
using dba::ProblemRange;

constexpr int kKernels = 4;   // local, consensus, norms, learned
constexpr int kGraphBatch = 16;
// timing mask bit: events only in the first iteration of a captured graph
constexpr unsigned kFirstOnly = 0x10u;

struct Buffers {
    std::vector<void *> ptrs;
    ~Buffers() { release(); }
    void release()
    {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
    template <typename T>
    hipError_t alloc(T **out, size_t count)
    {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return hipSuccess;
    }
};

struct ProblemSet {
    Buffers buf;
    int n_problems = 0;
    std::vector<ProblemRange> ranges;
    std::vector<int> m, n;
    std::vector<long long> L;
    DevArrays<float> a32{};
    DevArrays<double> a64{};
    uint8_t *mask = nullptr;
    long long n_slots = 0;
};

struct Timing {
    bool on = false;
    unsigned mask = 0xF;  // kernel ids timed (bit per id)
    double total_ms[kKernels] = {0, 0, 0, 0};
    long long launches[kKernels] = {0, 0, 0, 0};
    std::vector<hipEvent_t> pool;
    std::vector<int> pending_kernel;  // kernel id per recorded pair
    size_t used = 0;
};

// A captured graph of iterations whose kernels are bracketed by event-record
// nodes, for timed iterations on the graph path.  Two per graph size: one
// replay's times are read while the other replay runs.
struct TimedGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;  // two per kernel launch, in launch order
    std::vector<int> kid;        // kernel id per pair
    bool pending = false;        // launched, times not yet read
};

// The learned warm start's network on the device.
struct Mlp {
    Buffers buf;
    bool ready = false;
    __bf16 *w = nullptr;      // packed bf16 weights
    float *master = nullptr;  // FP32 parameters (kPTotal)
    float *norm = nullptr;    // kNormTotal
    float *xform = nullptr;   // [2][kIn] input scale and shift
    float *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    long long adam_t = 0;     // Adam steps taken since the moments were zeroed
    MlpParams params() const
    {
        return MlpParams{w, master + kPB1, master + kPB2, master + kPB3, norm, xform};
    }
};

}  // namespace host
}  // namespace dba

struct dba_handle {
    dba_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 256;
    std::string err;
    dba::host::ProblemSet *ps = nullptr;
    bool fp32 = false;
    dba::SolverParams sp{};
    // schedule
    int block_waves = 4, persistent = 0, tuned = 0;
    bool schedule_ready = false;
    int tune_next = 0;
    std::vector<float> tune_ms;
    // segment schedule of the point consensus (1 direct loads, 2 / 3 LDS tiles)
    int seg_sched = 1, seg_tuned = 0;
    bool seg_ready = false;
    int seg_next = 0;
    std::vector<float> seg_ms;
    // graphs: [0] one iteration, [1] kGraphBatch iterations
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    dba::host::Timing timing;
    // timed graphs [size as gexec][buffer]; off after a failed capture
    dba::host::TimedGraph tgraph[2][2];
    unsigned tgraph_mask = 0;  // the timing mask the timed graphs were captured with
    int tgraph_next[2] = {0, 0};
    bool tgraph_off = false;
    // sampled timing: [0] an iteration without its local launch, [1] that
    // and kGraphBatch - 1 more iterations; off after a failed capture
    hipGraphExec_t sgexec[2] = {nullptr, nullptr};
    bool sgraph_off = false;
    // learned warm start
    int start = DBA_START_PLAIN;
    dba::host::Mlp *mlp = nullptr;
    // this GPU's scratch array of the allocation-free entry point
    void *noalloc_scratch = nullptr;
};

namespace dba {
namespace host {

inline int fail(dba_handle *h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    return code;
}

#define HIP_TRY(h, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::dba::host::fail((h), DBA_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

void drop_graphs(dba_handle *h);
// Reads the kernel times of launches still pending (kernel timing mode).
int collect_timing(dba_handle *h);

}  // namespace host
}  // namespace dba
