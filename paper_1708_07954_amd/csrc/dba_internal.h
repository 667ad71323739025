// dba_internal.h -- device data layout and kernel launchers shared by the
// host runtime (dba_host.cpp) and the kernels (dba_kernels.hip,
// dba_block_kernels.hip).
//
// Layout of one problem set (one or many independent problems, concatenated
// with global camera / point / observation numbering):
//
//  * camera-major SLOTS: the observations of global camera J occupy slots
//    [cam_chunk0[J]*64, cam_chunk0[J]*64 + M_J), padded to a multiple of 64,
//    so every 64-slot CHUNK (one wavefront) belongs to exactly one camera.
//    Per slot (structure of arrays): uv (R2), pslot (point-major record index,
//    -1 for padding), ptid (global point), copy_y[9] (R), dual_y[9] (FP64).
//  * point-major RECORDS: the observations of global point I occupy records
//    [pt_off[I], pt_off[I+1]).  Per record: xrec (PtCopy: point copy x_i^j)
//    and urec (PtDual: point-side scaled dual).
//  * consensus: cons_y [n_cams][16] doubles (9 used), cons_x [n_points] double4.
//  * per-problem control block Ctrl (rho, pending dual rescale, residuals).
//
// One ADMM iteration = three launches:
//  local   : per slot, apply the previous iteration's dual update (deferred,
//            with the rho rescale), solve the local problem (Eq. 9) by robust
//            LM, write the copy, and emit per-chunk sums for the camera
//            consensus (copy_y + u_y, copy_y - cons_y, |copy_y - cons_y|^2);
//  consensus: point consensus (Eq. 10) from the records, camera consensus
//            (Eq. 11) from the chunk sums, residual partials;
//  norms   : per problem, primal/dual residuals and residual balancing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dba_layout.h"  // kChunk, kConsY, cons_group, ProblemRange

namespace dba {

constexpr int kCpart = 20;     // doubles per chunk partial: 9 sum(copy+u), 9 sum(d), 1 sum|d|^2, pad
constexpr int kEpart = 5;      // doubles per chunk of the reprojection statistics
constexpr int kNormThreads = 256;

struct Ctrl {
    double rho_x, rho_y;           // rho the next local solve uses
    double ratio_x, ratio_y;       // pending dual rescale rho_old / rho_new
    double last_rho_x, last_rho_y; // rho used by the last iteration
    double primal, dual;           // residuals of the last iteration
    double rb_mu, rb_tau, rho_min, rho_max;
    long long iteration;
    int pending;                   // 1: the last dual update (Eqs. 12-13) is not yet applied
    int nonfinite;
    int balancing;
    int pad[3];
};

template <typename R> struct Vec;
template <> struct Vec<float> { using R2 = float2; };
template <> struct Vec<double> { using R2 = double2; };

// Point record: the point copy x_i^j (local precision) and its scaled dual
// (FP64), three values each with no padding (12 / 24 and 24 bytes).
template <typename R> struct PtCopy { R x, y, z; };
struct PtDual { double x, y, z; };

template <typename R>
struct DevArrays {
    // slots
    long long n_slots;
    const typename Vec<R>::R2 *uv;
    const int *pslot;
    const int *ptid;
    R *copy_y;            // [9][n_slots]
    double *dual_y;       // [9][n_slots]
    int camera_blocks;    // 1: one camera copy per chunk (block local updates)
    R *copy_yc;           // [n_chunks][9] camera copy of the chunk (block local updates)
    double *dual_yc;      // [n_chunks][9] its scaled dual
    int n_blocks2;        // two-camera blocks (0: none): one wavefront each
    const int *blk_chunk; // [n_blocks2][2] chunk of the pair's first / second camera, or -1
    const int *blk_rec;   // [n_blocks2][64] point record of each lane, or -1
    const int *blk_cam;   // [n_blocks2][2] camera of the pair's first / second chunk, or -1
    const int *blk_prob;  // [n_blocks2] problem of the block
    const int *blk_pt;    // [n_blocks2][64] point of each lane, or -1
    const uint8_t *mask;  // [n_slots] evaluation mask
    const int *slot_orig; // [n_slots] observation index within its problem
    // records
    long long n_recs;
    PtCopy<R> *xrec;
    PtDual *urec;
    const int *pt_off;    // [n_pts+1]
    // chunks / cameras / points
    int n_chunks, n_cams, n_pts, n_problems;
    const int *chunk_cam;   // [n_chunks]
    const int *chunk_prob;  // [n_chunks] problem of the chunk (its camera's)
    const int *cam_prob;    // [n_cams]
    const int *pt_prob;     // [n_pts]
    const int *cam_chunk0;  // [n_cams+1]
    const int *cam_count;   // [n_cams]
    double *cons_y;         // [n_cams][16]
    double4 *cons_x;        // [n_pts]
    Ctrl *ctrl;             // [n_problems]
    const ProblemRange *prob; // [n_problems]
    double *cpart;          // [n_chunks][kCpart]
    int n_cw;
    const int *cw_pt0;      // [n_cw + 1] first global point of each consensus wave
    double *ppart;          // [n_cw / kConsWaves][2] workgroup sums of the point residual terms
    double *campart;        // [n_cams][2]
    double *epart;          // [n_chunks][kEpart]
    double *estats;         // [n_problems][kEpart]
};

struct SolverParams {
    int loss;
    double loss_param;
    int lm_steps;
    double lambda0;
    int learned_steps;   // LM steps after the learned start
    int camera;          // 0: angle-axis camera (9 parameters), 1: Euler camera (Eq. 1)
    int solver;          // 0: robust LM, 1: Gauss-Newton (per-observation local solves)
};

// ---- learned warm start: 26 -> 128 -> GELU -> 128 -> GELU -> 12 network
constexpr int kIn = 26, kInPad = 32, kHid = 128, kOut = 12, kOutPad = 16;
// packed bf16 weight block (dense, row-major):
//   W1^T [128][32] | W2^T [128][128] | W3^T [16][128] | W2 [128][128] | W3 [128][32]
constexpr int kOffW1T = 0;
constexpr int kOffW2T = kOffW1T + kHid * kInPad;
constexpr int kOffW3T = kOffW2T + kHid * kHid;
constexpr int kOffW2N = kOffW3T + kOutPad * kHid;
constexpr int kOffW3N = kOffW2N + kHid * kHid;
constexpr int kWTotal = kOffW3N + kHid * 2 * kOutPad;
// FP32 master parameters (flat): W1 [32][128] | b1 [128] | W2 [128][128] | b2 [128] | W3 [128][16] | b3 [16]
constexpr int kPW1 = 0, kPB1 = kPW1 + kInPad * kHid, kPW2 = kPB1 + kHid, kPB2 = kPW2 + kHid * kHid,
              kPW3 = kPB2 + kHid, kPB3 = kPW3 + kHid * kOutPad, kPTotal = kPB3 + kOutPad;
// normalisation block: mu_in[26] sd_in[26] mu_out[12] sd_out[12]
constexpr int kNormTotal = 2 * kIn + 2 * kOut;
// allocation-free network forward: rows per call and the scratch they need
// (standardised BF16 inputs and padded FP32 outputs)
constexpr long long kNoAllocMaxRows = 65536;
constexpr long long kNoAllocScratchBytes = kNoAllocMaxRows * (kInPad * 2 + kOutPad * 4);

struct MlpParams {
    const __bf16 *w;       // packed bf16 weights (kWTotal)
    const float *b1, *b2, *b3;
    const float *norm;     // kNormTotal
    const float *xform;    // [2][kIn]: 1 / sd_in, -mu_in / sd_in (input standardization)
};

// launchers (dba_kernels.hip; launch_local_block in dba_block_kernels.hip);
// each returns hipGetLastError()
template <typename R>
hipError_t launch_local(const DevArrays<R> &a, const SolverParams &sp, int block_waves,
                        int persistent, int n_cu, hipStream_t s);
hipError_t launch_local_learned(const DevArrays<float> &a, const SolverParams &sp, const MlpParams &mp,
                                int persistent, int n_cu, hipStream_t s);
template <typename R>
hipError_t launch_local_block(const DevArrays<R> &a, const SolverParams &sp, int block_waves, int persistent,
                              int n_cu, hipStream_t s);
template <typename R>
hipError_t launch_consensus(const DevArrays<R> &a, int schedule, hipStream_t s);

// network kernels (mlp_kernels.hip)
hipError_t mlp_pack(const float *P, __bf16 *w, hipStream_t s);
hipError_t mlp_prepare(const float *feat, const float *delta, const float *norm, long long n, __bf16 *xq, float *t,
                       hipStream_t s);
hipError_t mlp_forward(const __bf16 *xq, const int *rows, int n, const MlpParams &mp, float *y, __bf16 *xb, float *gp1,
                       __bf16 *h1, float *gp2, __bf16 *h2, hipStream_t s);
hipError_t mlp_backward(const float *y, const float *tq, const int *rows, int n, const __bf16 *w, const float *gp1,
                        const float *gp2, float *dy, __bf16 *dyq, float *dz2, __bf16 *dz2q, float *dz1, __bf16 *dz1q,
                        float *loss_part, hipStream_t s);
hipError_t mlp_wgrad(const __bf16 *xb, const __bf16 *h1, const __bf16 *h2, const __bf16 *dyq, const __bf16 *dz2q,
                     const __bf16 *dz1q, int n, float *grad, hipStream_t s);
hipError_t mlp_bias(const float *dy, const float *dz2, const float *dz1, int n, float *grad, hipStream_t s);
hipError_t mlp_adam(float *P, float *m, float *v, const float *g, float lr, float bc1, float bc2, hipStream_t s);
hipError_t mlp_destandardize(const float *y, const float *norm, long long n, float *delta, hipStream_t s);
hipError_t noalloc_scratch(int device, void **ptr);
hipError_t collect_pairs(const DevArrays<float> &a, const SolverParams &sp, const int *slots, int n, float *feat,
                         float *delta, int conv_steps, hipStream_t s);
template <typename R>
hipError_t launch_norms(const DevArrays<R> &a, hipStream_t s);
template <typename R>
hipError_t launch_eval(const DevArrays<R> &a, const SolverParams &sp, hipStream_t s);
template <typename R>
hipError_t launch_materialize(const DevArrays<R> &a, int problem, double *copies, double *duals,
                              hipStream_t s);

}  // namespace dba
