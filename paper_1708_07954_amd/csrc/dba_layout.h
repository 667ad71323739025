// dba_layout.h -- host-only construction of a problem set's device layout
// (no HIP types): validation of one problem's inputs and the slot / record /
// chunk arrays that dba_host.cpp uploads.  Built without a GPU toolchain too,
// so the CPU test suite runs it under AddressSanitizer and
// UndefinedBehaviorSanitizer.
//
// Layout (see dba_internal.h): camera-major 64-slot chunks (one camera per
// chunk), point-major records, consensus rows, per-problem index ranges.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "dba.h"

namespace dba {

constexpr int kChunk = 64;
constexpr int kConsY = 16;      // doubles per camera consensus row

// Point consensus order: a point's n records are summed in groups of
// cons_group(n) consecutive records (8, or n / 64 rounded up when n > 512, so
// that a point has at most 64 groups), each group in record order, and the
// group sums in group order.  The consensus waves below and every kernel
// schedule follow this order, so their results are bitwise identical.
constexpr int kGroupMin = 8;
constexpr int cons_group(int n) { return n > 64 * kGroupMin ? (n + 63) / 64 : kGroupMin; }
constexpr int cons_groups(int n) { return (n + cons_group(n) - 1) / cons_group(n); }
// consensus waves per workgroup of the consensus kernel; a problem's waves
// fill whole workgroups (the last ones may be empty), whose residual terms
// are summed per workgroup
constexpr int kConsWaves = 4;

struct ProblemRange {           // per problem, global index ranges
    int cam0, n_cams;
    int pt0, n_points;
    int chunk0, n_chunks;
    int cw0, n_cw;              // consensus waves (point ranges of the consensus kernel)
    long long rec0, n_obs;
};

// What of dba_options the layout depends on.
struct LayoutOptions {
    int camera_blocks = 0;      // one camera copy per chunk
    int block_points = 0;       // observations per one-camera block (0: 64)
    int block_cameras = 1;      // 2: two-camera blocks
    int camera_model = 0;       // 1: Euler camera (slots 6..8 checked)
};

// The host arrays of a problem set, R = float or double (local precision).
// Vector-typed device arrays are flattened: uv [n_slots][2], xrec
// [n_recs][3], cons_x [n_pts][4], cons_y [n_cams][kConsY].
template <typename R>
struct Layout {
    int n_problems = 0;
    std::vector<ProblemRange> ranges;
    long long n_slots = 0, n_chunks = 0, n_recs = 0;
    int n_cams = 0, n_pts = 0, n_cw = 0, n_blocks2 = 0;
    std::vector<R> uv;                      // [n_slots][2]
    std::vector<int> pslot, ptid, orig;     // [n_slots]; pslot -1 on padding
    std::vector<R> copy_y;                  // [9][n_slots] (per-observation local problems)
    std::vector<R> xrec;                    // [n_recs][3]
    std::vector<int> pt_off;                // [n_pts + 1]
    std::vector<int> chunk_cam, chunk_prob; // [n_chunks]: camera and problem of each chunk
    std::vector<int> cam_prob, cam_chunk0, cam_count;  // [n_cams] (+1 for cam_chunk0)
    std::vector<int> pt_prob;               // [n_pts]
    std::vector<double> cons_y;             // [n_cams][kConsY]
    std::vector<double> cons_x;             // [n_pts][4]
    std::vector<int> cw_pt0;                // [n_cw + 1] first point of each consensus wave: at
                                            // most 64 points with at most 64 record groups in
                                            // all, within one problem; n_cw a multiple of
                                            // kConsWaves per problem
    std::vector<int> blk_chunk, blk_rec;    // two-camera blocks: [n_blocks2][2], [n_blocks2][64]
    std::vector<int> blk_cam, blk_prob;     // two-camera blocks: camera of each chunk (or -1), problem
    std::vector<int> blk_pt;                // two-camera blocks: point of each lane (or -1)
    std::vector<R> copy_yc;                 // [n_chunks][9] camera copy per chunk
};

// Validates problem p's inputs (sizes, indices, finite values, every camera
// and point observed, positive depth at the start).  Returns DBA_OK or the
// status with a message in *err.
int validate_problem(int p, const dba_problem_desc &d, int camera_model, std::string *err);

// Builds the layout of np problems.  Returns DBA_OK, or DBA_E_INVALID_ARG
// with a message in *err (a camera observing a point twice with two-camera
// blocks, or a set too large for 32-bit slot indexes).
template <typename R>
int build_layout(const LayoutOptions &o, int np, const dba_problem_desc *probs, Layout<R> *out, std::string *err);

}  // namespace dba
