// dba_learned.cpp -- C ABI of the learned warm start: the network's
// parameters, batch evaluation, loss gradient, collection of training pairs
// from plain iterations, and training with Adam on the GPU kernels of
// mlp_kernels.hip.
#include "dba_host_internal.h"

#include <cmath>
#include <cstring>

using namespace dba::host;

namespace {

uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &st) { return (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); }

int ensure_mlp(dba_handle *h)
{
    if (h->mlp) return DBA_OK;
    Mlp *m = new Mlp();
    HIP_TRY(h, m->buf.alloc(&m->w, dba::kWTotal));
    HIP_TRY(h, m->buf.alloc(&m->master, dba::kPTotal));
    HIP_TRY(h, m->buf.alloc(&m->norm, dba::kNormTotal));
    HIP_TRY(h, m->buf.alloc(&m->xform, 2 * dba::kIn));
    HIP_TRY(h, m->buf.alloc(&m->adam_m, dba::kPTotal));
    HIP_TRY(h, m->buf.alloc(&m->adam_v, dba::kPTotal));
    HIP_TRY(h, m->buf.alloc(&m->grad, dba::kPTotal));
    h->mlp = m;
    return DBA_OK;
}

int upload_mlp(dba_handle *h, const float *params, const float *norm)
{
    int rc = ensure_mlp(h);
    if (rc != DBA_OK) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->mlp->master, params, dba::kPTotal * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->mlp->norm, norm, dba::kNormTotal * sizeof(float), hipMemcpyHostToDevice, h->stream));
    float xf[2 * dba::kIn];
    for (int k = 0; k < dba::kIn; ++k) {
        xf[k] = 1.0f / norm[dba::kIn + k];
        xf[dba::kIn + k] = -norm[k] / norm[dba::kIn + k];
    }
    HIP_TRY(h, hipMemcpyAsync(h->mlp->xform, xf, sizeof(xf), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, dba::mlp_pack(h->mlp->master, h->mlp->w, h->stream));
    // a new network starts its optimiser state from zero
    HIP_TRY(h, hipMemsetAsync(h->mlp->adam_m, 0, dba::kPTotal * sizeof(float), h->stream));
    HIP_TRY(h, hipMemsetAsync(h->mlp->adam_v, 0, dba::kPTotal * sizeof(float), h->stream));
    h->mlp->adam_t = 0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->mlp->ready = true;
    drop_graphs(h);
    return DBA_OK;
}

// One Adam step (bias-corrected, step counter t + 1) of the master
// parameters with the gradient already in M.grad, then the bf16 weights.
int adam_step(dba_handle *h, double lr)
{
    Mlp &M = *h->mlp;
    const long long t = ++M.adam_t;
    const double bc1 = 1.0 - std::pow(0.9, (double)t), bc2 = 1.0 - std::pow(0.999, (double)t);
    HIP_TRY(h, dba::mlp_adam(M.master, M.adam_m, M.adam_v, M.grad, (float)lr, (float)bc1, (float)bc2, h->stream));
    HIP_TRY(h, dba::mlp_pack(M.master, M.w, h->stream));
    return DBA_OK;
}

// Sets the local start; cached graphs (plain and timed) are captured with
// one start's kernel, so a change reads pending kernel times and drops them.
int switch_start(dba_handle *h, int start)
{
    if (h->start == start) return DBA_OK;
    const int rc = collect_timing(h);
    drop_graphs(h);
    h->start = start;
    return rc;
}

}  // namespace

namespace dba {
namespace host {
void free_mlp(dba_handle *h)
{
    delete h->mlp;
    h->mlp = nullptr;
}
}  // namespace host
}  // namespace dba

extern "C" {

int dba_set_mlp(dba_handle *h, const float *params, const float *norm)
{
    if (!h || !params || !norm) return DBA_E_INVALID_ARG;
    h->err.clear();
    for (int q = 0; q < dba::kPTotal; ++q)
        if (!std::isfinite(params[q])) return fail(h, DBA_E_NONFINITE, "network parameter %d not finite", q);
    for (int q = 0; q < dba::kNormTotal; ++q)
        if (!std::isfinite(norm[q]) || (((q >= dba::kIn && q < 2 * dba::kIn) || q >= 2 * dba::kIn + dba::kOut) && !(norm[q] > 0)))
            return fail(h, DBA_E_INVALID_ARG, "normalisation entry %d invalid", q);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    return upload_mlp(h, params, norm);
}

int dba_get_mlp(dba_handle *h, float *params, float *norm)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    if (params)
        HIP_TRY(h, hipMemcpyAsync(params, h->mlp->master, dba::kPTotal * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (norm)
        HIP_TRY(h, hipMemcpyAsync(norm, h->mlp->norm, dba::kNormTotal * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return DBA_OK;
}

int dba_set_start(dba_handle *h, int32_t start, int32_t learned_lm_steps)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (start != DBA_START_PLAIN && start != DBA_START_LEARNED) return fail(h, DBA_E_INVALID_ARG, "bad start %d", start);
    if (learned_lm_steps < 0 || learned_lm_steps > 64) return fail(h, DBA_E_INVALID_ARG, "bad learned_lm_steps");
    if (start == DBA_START_LEARNED && !h->fp32)
        return fail(h, DBA_E_INVALID_ARG, "the learned start runs with FP32 local solves");
    if (start == DBA_START_LEARNED && h->opt.camera_blocks)
        return fail(h, DBA_E_INVALID_ARG, "the learned start is for one observation per local problem");
    h->sp.learned_steps = learned_lm_steps;
    const int rc = collect_timing(h);
    drop_graphs(h);
    h->start = start;
    return rc;
}

int dba_mlp_forward(dba_handle *h, const float *features, int64_t n, float *delta)
{
    if (!h || !features || !delta || n < 1 || n > (1LL << 28)) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    Buffers B;
    float *df, *dy;
    __bf16 *xq;
    HIP_TRY(h, B.alloc(&df, n * dba::kIn));
    HIP_TRY(h, B.alloc(&xq, n * dba::kInPad));
    HIP_TRY(h, B.alloc(&dy, n * dba::kOutPad));
    HIP_TRY(h, hipMemcpyAsync(df, features, n * dba::kIn * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, dba::mlp_prepare(df, nullptr, h->mlp->norm, n, xq, nullptr, h->stream));
    HIP_TRY(h, dba::mlp_forward(xq, nullptr, (int)n, h->mlp->params(), dy, nullptr, nullptr, nullptr, nullptr, nullptr,
                                h->stream));
    std::vector<float> y(n * dba::kOutPad), nm(dba::kNormTotal);
    HIP_TRY(h, hipMemcpyAsync(y.data(), dy, y.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(nm.data(), h->mlp->norm, nm.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int64_t r = 0; r < n; ++r)
        for (int o = 0; o < dba::kOut; ++o)
            delta[r * dba::kOut + o] = y[r * dba::kOutPad + o] * nm[2 * dba::kIn + dba::kOut + o] + nm[2 * dba::kIn + o];
    return DBA_OK;
}

static_assert(DBA_NOALLOC_MAX_ROWS == dba::kNoAllocMaxRows && DBA_NOALLOC_SCRATCH_BYTES == dba::kNoAllocScratchBytes,
              "the header's scratch limits match the library's");

int dba_mlp_forward_noalloc(dba_handle *h, const float *features, int64_t n, float *delta)
{
    if (!h || !features || !delta || n < 1) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (n > dba::kNoAllocMaxRows)
        return fail(h, DBA_E_INVALID_ARG, "%lld rows exceed the %lld of the scratch array", (long long)n,
                    dba::kNoAllocMaxRows);
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    if (!h->noalloc_scratch) return fail(h, DBA_E_STATE, "no scratch address for this device");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    // every byte read below is written first by the same call: the inputs
    // for rows < n by the prepare kernel, the outputs for rows < n by the
    // forward kernel
    __bf16 *xq = static_cast<__bf16 *>(h->noalloc_scratch);
    float *dy = reinterpret_cast<float *>(static_cast<unsigned char *>(h->noalloc_scratch) +
                                          dba::kNoAllocMaxRows * dba::kInPad * sizeof(__bf16));
    HIP_TRY(h, dba::mlp_prepare(features, nullptr, h->mlp->norm, n, xq, nullptr, h->stream));
    HIP_TRY(h, dba::mlp_forward(xq, nullptr, (int)n, h->mlp->params(), dy, nullptr, nullptr, nullptr, nullptr, nullptr,
                                h->stream));
    HIP_TRY(h, dba::mlp_destandardize(dy, h->mlp->norm, n, delta, h->stream));
    return DBA_OK;
}

int dba_mlp_loss_grad(dba_handle *h, const float *x_std, const float *t_std, int32_t n, float *loss, float *grad,
                      float *y_out)
{
    if (!h || !x_std || !t_std || n < 64 || n % 64 || n > 65536) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    Buffers B;
    std::vector<__bf16> xh((size_t)n * dba::kInPad);
    for (size_t q = 0; q < xh.size(); ++q) xh[q] = (__bf16)x_std[q];
    __bf16 *xq, *xb, *h1, *h2, *dyq, *dz2q, *dz1q;
    float *t, *y, *gp1, *gp2, *dy, *dz2, *dz1, *lp;
    HIP_TRY(h, B.alloc(&xq, (size_t)n * dba::kInPad));
    HIP_TRY(h, B.alloc(&xb, (size_t)n * dba::kInPad));
    HIP_TRY(h, B.alloc(&t, (size_t)n * dba::kOutPad));
    HIP_TRY(h, B.alloc(&y, (size_t)n * dba::kOutPad));
    HIP_TRY(h, B.alloc(&gp1, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&gp2, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&h1, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&h2, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&dy, (size_t)n * dba::kOutPad));
    HIP_TRY(h, B.alloc(&dyq, (size_t)n * 2 * dba::kOutPad));
    HIP_TRY(h, B.alloc(&dz2, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&dz1, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&dz2q, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&dz1q, (size_t)n * dba::kHid));
    HIP_TRY(h, B.alloc(&lp, n / 64));
    HIP_TRY(h, hipMemcpyAsync(xq, xh.data(), xh.size() * sizeof(__bf16), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(t, t_std, (size_t)n * dba::kOutPad * sizeof(float), hipMemcpyHostToDevice, h->stream));
    const dba::MlpParams mp = h->mlp->params();
    HIP_TRY(h, dba::mlp_forward(xq, nullptr, n, mp, y, xb, gp1, h1, gp2, h2, h->stream));
    HIP_TRY(h, dba::mlp_backward(y, t, nullptr, n, mp.w, gp1, gp2, dy, dyq, dz2, dz2q, dz1, dz1q, lp, h->stream));
    HIP_TRY(h, hipMemsetAsync(h->mlp->grad, 0, dba::kPTotal * sizeof(float), h->stream));
    HIP_TRY(h, dba::mlp_wgrad(xb, h1, h2, dyq, dz2q, dz1q, n, h->mlp->grad, h->stream));
    HIP_TRY(h, dba::mlp_bias(dy, dz2, dz1, n, h->mlp->grad, h->stream));
    std::vector<float> l(n / 64);
    HIP_TRY(h, hipMemcpyAsync(l.data(), lp, l.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (grad)
        HIP_TRY(h, hipMemcpyAsync(grad, h->mlp->grad, dba::kPTotal * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (y_out)
        HIP_TRY(h, hipMemcpyAsync(y_out, y, (size_t)n * dba::kOutPad * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    double s = 0.0;
    for (float v : l) s += v;
    if (loss) *loss = (float)(s / ((double)n * dba::kOut));
    return DBA_OK;
}

int dba_mlp_apply_gradient(dba_handle *h, const float *grad, double lr)
{
    if (!h || !grad || !(lr > 0) || !std::isfinite(lr)) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    for (int q = 0; q < dba::kPTotal; ++q)
        if (!std::isfinite(grad[q])) return fail(h, DBA_E_NONFINITE, "gradient entry %d not finite", q);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, hipMemcpyAsync(h->mlp->grad, grad, dba::kPTotal * sizeof(float), hipMemcpyHostToDevice, h->stream));
    const int rc = adam_step(h, lr);
    if (rc != DBA_OK) return rc;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    return DBA_OK;
}

int dba_mlp_adam_state(dba_handle *h, float *m, float *v, int64_t *step)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->mlp || !h->mlp->ready) return fail(h, DBA_E_STATE, "no network set");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    if (m) HIP_TRY(h, hipMemcpyAsync(m, h->mlp->adam_m, dba::kPTotal * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    if (v) HIP_TRY(h, hipMemcpyAsync(v, h->mlp->adam_v, dba::kPTotal * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (step) *step = h->mlp->adam_t;
    return DBA_OK;
}

int dba_collect_pairs(dba_handle *h, int32_t n_iters, int32_t per_iter, uint64_t seed, int32_t conv_steps,
                      float *features, float *deltas)
{
    if (!h || n_iters < 1 || per_iter < 1 || conv_steps < 1 || conv_steps > 200 || !features || !deltas)
        return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->ps) return fail(h, DBA_E_STATE, "no problem set");
    if (!h->fp32) return fail(h, DBA_E_INVALID_ARG, "pairs are collected from FP32 local solves");
    if (h->opt.camera_blocks)
        return fail(h, DBA_E_INVALID_ARG, "pairs are collected from per-observation local solves");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    ProblemSet &ps = *h->ps;
    std::vector<int> pslot(ps.n_slots), active;
    HIP_TRY(h, hipMemcpy(pslot.data(), ps.a32.pslot, ps.n_slots * sizeof(int), hipMemcpyDeviceToHost));
    for (long long q = 0; q < ps.n_slots; ++q)
        if (pslot[q] >= 0) active.push_back((int)q);
    Buffers B;
    int *dslots;
    float *df, *dd;
    HIP_TRY(h, B.alloc(&dslots, per_iter));
    HIP_TRY(h, B.alloc(&df, (size_t)per_iter * dba::kIn));
    HIP_TRY(h, B.alloc(&dd, (size_t)per_iter * dba::kOut));
    std::vector<int> pick(per_iter);
    uint64_t st = seed;
    const int saved = h->start;
    // the captured graphs hold the local kernel of the start they were
    // captured with: switching the start drops them, both ways
    int rc0 = switch_start(h, DBA_START_PLAIN);
    if (rc0 != DBA_OK) return rc0;
    for (int it = 0; it < n_iters; ++it) {
        for (int q = 0; q < per_iter; ++q) pick[q] = active[(size_t)(uniform01(st) * active.size()) % active.size()];
        HIP_TRY(h, hipMemcpyAsync(dslots, pick.data(), per_iter * sizeof(int), hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, dba::collect_pairs(ps.a32, h->sp, dslots, per_iter, df, dd, conv_steps, h->stream));
        HIP_TRY(h, hipMemcpyAsync(features + (size_t)it * per_iter * dba::kIn, df, (size_t)per_iter * dba::kIn * sizeof(float),
                                  hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipMemcpyAsync(deltas + (size_t)it * per_iter * dba::kOut, dd, (size_t)per_iter * dba::kOut * sizeof(float),
                                  hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        const int rc = dba_iterate(h, 1);
        if (rc != DBA_OK) {
            (void)switch_start(h, saved);
            return rc;
        }
    }
    rc0 = switch_start(h, saved);
    if (rc0 != DBA_OK) return rc0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    return DBA_OK;
}

int dba_mlp_train(dba_handle *h, const float *features, const float *deltas, int64_t n, int32_t epochs, int32_t batch,
                  double lr, uint64_t seed, float *epoch_loss)
{
    if (!h || !features || !deltas || epochs < 1 || batch < 64 || batch % 64 || batch > 65536 || n < batch ||
        n > (1LL << 28) || !(lr > 0))
        return DBA_E_INVALID_ARG;
    h->err.clear();
    HIP_TRY(h, hipSetDevice(h->opt.device));
    // standardisation statistics
    std::vector<float> norm(dba::kNormTotal);
    for (int k = 0; k < dba::kIn + dba::kOut; ++k) {
        const float *src = k < dba::kIn ? features + k : deltas + (k - dba::kIn);
        const int ld = k < dba::kIn ? dba::kIn : dba::kOut;
        double s = 0.0, s2 = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            const double x = src[r * ld];
            if (!std::isfinite(x)) return fail(h, DBA_E_NONFINITE, "training pair %lld not finite", (long long)r);
            s += x;
            s2 += x * x;
        }
        const double mu = s / n, var = std::max(s2 / n - mu * mu, 0.0), sd = std::sqrt(var);
        const int mi = k < dba::kIn ? k : 2 * dba::kIn + (k - dba::kIn);
        const int si = k < dba::kIn ? dba::kIn + k : 2 * dba::kIn + dba::kOut + (k - dba::kIn);
        norm[mi] = (float)mu;
        norm[si] = sd > 1e-20 ? (float)sd : 1.0f;
    }
    // initial parameters: N(0, 1/fan_in), zero biases and padding
    std::vector<float> P(dba::kPTotal, 0.0f);
    uint64_t st = seed ^ 0x5DEECE66DULL;
    auto gauss = [&]() {
        const double u1 = std::max(uniform01(st), 1e-300), u2 = uniform01(st);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    for (int k = 0; k < dba::kIn; ++k)
        for (int u = 0; u < dba::kHid; ++u) P[dba::kPW1 + k * dba::kHid + u] = (float)(gauss() / std::sqrt((double)dba::kIn));
    for (int q = 0; q < dba::kHid * dba::kHid; ++q) P[dba::kPW2 + q] = (float)(gauss() / std::sqrt((double)dba::kHid));
    for (int k = 0; k < dba::kHid; ++k)
        for (int o = 0; o < dba::kOut; ++o) P[dba::kPW3 + k * dba::kOutPad + o] = (float)(gauss() / std::sqrt((double)dba::kHid));
    int rc = upload_mlp(h, P.data(), norm.data());
    if (rc != DBA_OK) return rc;
    Mlp &M = *h->mlp;
    // device data
    Buffers B;
    float *dfeat, *ddel, *t, *y, *gp1, *gp2, *dy, *dz2, *dz1, *lp;
    __bf16 *xq, *xb, *h1, *h2, *dyq, *dz2q, *dz1q;
    int *rows;
    const int steps = (int)(n / batch), tiles = batch / 64;
    HIP_TRY(h, B.alloc(&dfeat, n * dba::kIn));
    HIP_TRY(h, B.alloc(&ddel, n * dba::kOut));
    HIP_TRY(h, B.alloc(&xq, n * dba::kInPad));
    HIP_TRY(h, B.alloc(&t, n * dba::kOutPad));
    HIP_TRY(h, B.alloc(&rows, n));
    HIP_TRY(h, B.alloc(&y, (size_t)batch * dba::kOutPad));
    HIP_TRY(h, B.alloc(&xb, (size_t)batch * dba::kInPad));
    HIP_TRY(h, B.alloc(&gp1, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&gp2, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&h1, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&h2, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&dy, (size_t)batch * dba::kOutPad));
    HIP_TRY(h, B.alloc(&dyq, (size_t)batch * 2 * dba::kOutPad));
    HIP_TRY(h, B.alloc(&dz2, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&dz1, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&dz2q, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&dz1q, (size_t)batch * dba::kHid));
    HIP_TRY(h, B.alloc(&lp, (size_t)steps * tiles));
    HIP_TRY(h, hipMemcpyAsync(dfeat, features, n * dba::kIn * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(ddel, deltas, n * dba::kOut * sizeof(float), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, dba::mlp_prepare(dfeat, ddel, M.norm, n, xq, t, h->stream));
    HIP_TRY(h, hipMemsetAsync(M.grad, 0, dba::kPTotal * sizeof(float), h->stream));
    std::vector<int> perm(n);
    std::vector<float> lh((size_t)steps * tiles);
    const dba::MlpParams mp = M.params();
    const long long total = (long long)epochs * steps;
    long long step = 0;
    for (int e = 0; e < epochs; ++e) {
        for (int64_t q = 0; q < n; ++q) perm[q] = (int)q;
        uint64_t ps = seed + 0x1000 * (uint64_t)(e + 1);
        for (int64_t q = n - 1; q > 0; --q) {
            const int64_t r = (int64_t)(uniform01(ps) * (double)(q + 1)) % (q + 1);
            std::swap(perm[q], perm[r]);
        }
        HIP_TRY(h, hipMemcpyAsync(rows, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, h->stream));
        for (int s = 0; s < steps; ++s) {
            const int *rp = rows + (size_t)s * batch;
            HIP_TRY(h, dba::mlp_forward(xq, rp, batch, mp, y, xb, gp1, h1, gp2, h2, h->stream));
            HIP_TRY(h, dba::mlp_backward(y, t, rp, batch, M.w, gp1, gp2, dy, dyq, dz2, dz2q, dz1, dz1q,
                                         lp + (size_t)s * tiles, h->stream));
            HIP_TRY(h, dba::mlp_wgrad(xb, h1, h2, dyq, dz2q, dz1q, batch, M.grad, h->stream));
            HIP_TRY(h, dba::mlp_bias(dy, dz2, dz1, batch, M.grad, h->stream));
            ++step;
            const double lr_t = lr * 0.5 * (1.0 + std::cos(M_PI * (double)(step - 1) / (double)total));
            rc = adam_step(h, lr_t);
            if (rc != DBA_OK) return rc;
        }
        HIP_TRY(h, hipMemcpyAsync(lh.data(), lp, lh.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        double sl = 0.0;
        for (float v : lh) sl += v;
        if (epoch_loss) epoch_loss[e] = (float)(sl / ((double)steps * batch * dba::kOut));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    drop_graphs(h);
    return DBA_OK;
}

}  // extern "C"
