// dba_internal.h -- device data layout and kernel launchers shared by the
// host runtime (dba_host.cpp) and the kernels (dba_kernels.hip).
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
//    [pt_off[I], pt_off[I+1]).  Per record: xrec (R4: point copy x_i^j) and
//    urec (double4: point-side scaled dual).
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

namespace dba {

constexpr int kChunk = 64;
constexpr int kCpart = 20;     // doubles per chunk partial: 9 sum(copy+u), 9 sum(d), 1 sum|d|^2, pad
constexpr int kConsY = 16;     // doubles per camera consensus row
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

struct ProblemRange {              // per problem, global index ranges
    int cam0, n_cams;
    int pt0, n_points;
    int chunk0, n_chunks;
    int pblk0, n_pblk;             // point blocks of the consensus kernel
    long long rec0, n_obs;
};

constexpr int kPtBlock = 256;      // points per consensus block (never straddles problems)

template <typename R> struct Vec;
template <> struct Vec<float> { using R2 = float2; using R4 = float4; };
template <> struct Vec<double> { using R2 = double2; using R4 = double4; };

template <typename R>
struct DevArrays {
    // slots
    long long n_slots;
    const typename Vec<R>::R2 *uv;
    const int *pslot;
    const int *ptid;
    R *copy_y;            // [9][n_slots]
    double *dual_y;       // [9][n_slots]
    const uint8_t *mask;  // [n_slots] evaluation mask
    const int *slot_orig; // [n_slots] observation index within its problem
    // records
    long long n_recs;
    typename Vec<R>::R4 *xrec;
    double4 *urec;
    const int *pt_off;    // [n_pts+1]
    // chunks / cameras / points
    int n_chunks, n_cams, n_pts, n_problems;
    const int *chunk_cam;   // [n_chunks]
    const int *cam_prob;    // [n_cams]
    const int *pt_prob;     // [n_pts]
    const int *cam_chunk0;  // [n_cams+1]
    const int *cam_count;   // [n_cams]
    double *cons_y;         // [n_cams][16]
    double4 *cons_x;        // [n_pts]
    Ctrl *ctrl;             // [n_problems]
    const ProblemRange *prob; // [n_problems]
    double *cpart;          // [n_chunks][kCpart]
    int n_pblk;
    const int *pblk_pt0;    // [n_pblk] first global point of the block
    const int *pblk_cnt;    // [n_pblk] points in the block (<= kPtBlock)
    double *ppart;          // [n_pblk][2] block sums of the point residual terms
    double *campart;        // [n_cams][2]
    double *epart;          // [n_chunks][kEpart]
    double *estats;         // [n_problems][kEpart]
};

struct SolverParams {
    int loss;
    double loss_param;
    int lm_steps;
    double lambda0;
};

// launchers (dba_kernels.hip); each returns hipGetLastError()
template <typename R>
hipError_t launch_local(const DevArrays<R> &a, const SolverParams &sp, int block_waves,
                        int persistent, int n_cu, hipStream_t s);
template <typename R>
hipError_t launch_consensus(const DevArrays<R> &a, hipStream_t s);
template <typename R>
hipError_t launch_norms(const DevArrays<R> &a, hipStream_t s);
template <typename R>
hipError_t launch_eval(const DevArrays<R> &a, const SolverParams &sp, hipStream_t s);
template <typename R>
hipError_t launch_materialize(const DevArrays<R> &a, int problem, double *copies, double *duals,
                              hipStream_t s);

}  // namespace dba
