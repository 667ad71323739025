// dba_layout.cpp -- host-only layout builder and input validation (see
// dba_layout.h).  Plain C++: no HIP headers, so it also builds with g++ and
// the sanitizers on a machine without a GPU toolchain.
#include "dba_layout.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace dba {
namespace {

int set_err(std::string *err, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (err) *err = buf;
    return code;
}

// Depth P_3 of R(w) X + t (Rodrigues, series for small angles).
double depth_angle_axis(const double *cam, const double *X)
{
    const double w0 = cam[0], w1 = cam[1], w2 = cam[2];
    const double t2 = w0 * w0 + w1 * w1 + w2 * w2;
    double c, a, b;
    if (t2 < 1e-4) {
        c = 1.0 - t2 / 2.0 + t2 * t2 / 24.0;
        a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
        b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
    } else {
        const double t = std::sqrt(t2), sh = std::sin(0.5 * t);
        c = std::cos(t);
        a = std::sin(t) / t;
        b = 2.0 * sh * sh / t2;
    }
    const double wd = w0 * X[0] + w1 * X[1] + w2 * X[2];
    return c * X[2] + a * (w0 * X[1] - w1 * X[0]) + b * wd * w2 + cam[5];
}

// Depth P_3 of R X + t for the Euler camera, R = R3(gamma) R2(beta) R1(alpha):
// the third row of R is (-sin beta, sin alpha cos beta, cos alpha cos beta).
double depth_euler(const double *cam, const double *X)
{
    const double sa = std::sin(cam[0]), ca = std::cos(cam[0]), sb = std::sin(cam[1]), cb = std::cos(cam[1]);
    return -sb * X[0] + sa * cb * X[1] + ca * cb * X[2] + cam[5];
}

// Two-camera blocks of one problem (block_cameras == 2): cameras in pairs
// (2g, 2g + 1); a pair's observed points, ascending, in runs of at most bp
// points; block b holds run b with one copy of each of its points (lane l <->
// point pts[pts0[b] + l]) and of each pair camera s that observes one of them
// (bit s of present[b]); obs[(pts0[b] + l) * 2 + s] is the observation of
// camera s of the pair at lane l, or -1.  Returns false on a repeated
// (camera, point) pair, which a lane cannot hold.
struct PairBlocks {
    std::vector<int> cam0, npts, pts0, present, pts;
    std::vector<long long> obs;
};

bool pair_blocks(const dba_problem_desc &d, int bp, PairBlocks &out)
{
    const int ng = (d.n_cams + 1) / 2;
    std::vector<long long> goff(ng + 1, 0);
    for (long long k = 0; k < d.n_obs; ++k) ++goff[d.obs_cam[k] / 2 + 1];
    for (int g = 0; g < ng; ++g) goff[g + 1] += goff[g];
    std::vector<long long> gobs(d.n_obs), fill(goff.begin(), goff.end() - 1);
    for (long long k = 0; k < d.n_obs; ++k) gobs[fill[d.obs_cam[k] / 2]++] = k;
    std::vector<int> lane_of(d.n_points, -1);
    for (int g = 0; g < ng; ++g) {
        std::vector<int> gp;
        for (long long q = goff[g]; q < goff[g + 1]; ++q) gp.push_back(d.obs_point[gobs[q]]);
        std::sort(gp.begin(), gp.end());
        gp.erase(std::unique(gp.begin(), gp.end()), gp.end());
        const size_t first = out.pts.size();
        for (size_t r0 = 0; r0 < gp.size(); r0 += bp) {
            const int n = (int)std::min<size_t>(bp, gp.size() - r0);
            out.cam0.push_back(2 * g);
            out.npts.push_back(n);
            out.pts0.push_back((int)out.pts.size());
            out.present.push_back(0);
            for (int l = 0; l < n; ++l) {
                out.pts.push_back(gp[r0 + l]);
                out.obs.push_back(-1);
                out.obs.push_back(-1);
            }
        }
        for (size_t t = first; t < out.pts.size(); ++t) lane_of[out.pts[t]] = (int)t;
        // each observation of the pair into its point's lane
        for (long long q = goff[g]; q < goff[g + 1]; ++q) {
            const long long k = gobs[q];
            const int t = lane_of[d.obs_point[k]], sc = d.obs_cam[k] - 2 * g;
            if (out.obs[2 * (size_t)t + sc] >= 0) return false;
            out.obs[2 * (size_t)t + sc] = k;
        }
    }
    // presence bits, per block from its lanes
    for (size_t b = 0; b < out.cam0.size(); ++b)
        for (int l = 0; l < out.npts[b]; ++l)
            for (int sc = 0; sc < 2; ++sc)
                if (out.obs[2 * (size_t)(out.pts0[b] + l) + sc] >= 0) out.present[b] |= 1 << sc;
    return true;
}

}  // namespace

int validate_problem(int p, const dba_problem_desc &d, int camera_model, std::string *err)
{
    if (d.n_cams < 1 || d.n_points < 1 || d.n_obs < 1)
        return set_err(err, DBA_E_INVALID_ARG, "problem %d: sizes must be positive (m=%d n=%d L=%lld)", p,
                       d.n_cams, d.n_points, (long long)d.n_obs);
    if (!d.obs_cam || !d.obs_point || !d.obs_uv || !d.cams || !d.points)
        return set_err(err, DBA_E_INVALID_ARG, "problem %d: null array", p);
    if (d.n_obs > (1LL << 30))
        return set_err(err, DBA_E_INVALID_ARG, "problem %d: too many observations", p);
    std::vector<int> cc(d.n_cams, 0), pc(d.n_points, 0);
    for (long long k = 0; k < d.n_obs; ++k) {
        const int j = d.obs_cam[k], i = d.obs_point[k];
        if (j < 0 || j >= d.n_cams || i < 0 || i >= d.n_points)
            return set_err(err, DBA_E_INDEX_RANGE,
                           "problem %d: observation %lld has camera %d / point %d out of range", p, k, j, i);
        ++cc[j];
        ++pc[i];
        if (!std::isfinite(d.obs_uv[2 * k]) || !std::isfinite(d.obs_uv[2 * k + 1]))
            return set_err(err, DBA_E_NONFINITE, "problem %d: observation %lld is not finite", p, k);
    }
    for (long long q = 0; q < 9LL * d.n_cams; ++q)
        if (!std::isfinite(d.cams[q]))
            return set_err(err, DBA_E_NONFINITE, "problem %d: camera value %lld not finite", p, q);
    for (long long q = 0; q < 3LL * d.n_points; ++q)
        if (!std::isfinite(d.points[q]))
            return set_err(err, DBA_E_NONFINITE, "problem %d: point value %lld not finite", p, q);
    for (int j = 0; j < d.n_cams; ++j)
        if (!cc[j]) return set_err(err, DBA_E_UNOBSERVED, "problem %d: camera %d has no observation", p, j);
    for (int i = 0; i < d.n_points; ++i)
        if (!pc[i]) return set_err(err, DBA_E_UNOBSERVED, "problem %d: point %d has no observation", p, i);
    const bool euler = camera_model == 1;
    if (euler)
        for (int j = 0; j < d.n_cams; ++j) {
            const double *c = d.cams + 9LL * j;
            if (!(c[6] > 0) || c[7] != 0.0 || c[8] != 0.0)
                return set_err(err, DBA_E_INVALID_ARG,
                               "problem %d: camera %d: the Euler camera needs a focal length > 0 in slot 6 and "
                               "zeros in slots 7, 8", p, j);
        }
    for (long long k = 0; k < d.n_obs; ++k) {
        const double *cam = d.cams + 9LL * d.obs_cam[k], *X = d.points + 3LL * d.obs_point[k];
        const double z = euler ? depth_euler(cam, X) : depth_angle_axis(cam, X);
        if (!(z > 1e-6))
            return set_err(err, DBA_E_BEHIND_CAMERA, "problem %d: observation %lld has depth %g at the initial "
                           "estimate", p, k, z);
    }
    return DBA_OK;
}

template <typename R>
int build_layout(const LayoutOptions &o, int np, const dba_problem_desc *probs, Layout<R> *outp, std::string *err)
{
    Layout<R> &out = *outp;
    const int CH = kChunk;
    // observations of a camera per chunk: 64, or the block size pi of the
    // block local updates (the rest of such a chunk is padding).  Block local
    // updates keep the camera copy per chunk (copy_yc) and have no per-slot
    // camera copies (copy_y).
    const int BP = o.camera_blocks && o.block_points ? o.block_points : CH;
    const bool per_obs = !o.camera_blocks;
    // two-camera blocks: a point copy per (block, point), not per observation
    const bool k2 = o.camera_blocks && o.block_cameras == 2;
    std::vector<PairBlocks> pbs(k2 ? np : 0);
    // global sizes
    long long n_chunks = 0, n_recs = 0;
    int n_cams = 0, n_pts = 0, n_blocks = 0;
    out.n_problems = np;
    out.ranges.clear();
    out.cw_pt0.clear();
    for (int p = 0; p < np; ++p) {
        const dba_problem_desc &d = probs[p];
        std::vector<int> cc(d.n_cams, 0);
        for (long long k = 0; k < d.n_obs; ++k) ++cc[d.obs_cam[k]];
        ProblemRange r{};
        r.cam0 = n_cams; r.n_cams = d.n_cams;
        r.pt0 = n_pts; r.n_points = d.n_points;
        r.chunk0 = (int)n_chunks;
        long long ch = 0, nrec = d.n_obs;
        if (k2) {
            if (!pair_blocks(d, BP, pbs[p]))
                return set_err(err, DBA_E_INVALID_ARG, "problem %d: a camera observes a point twice (two-camera "
                               "blocks hold one observation per camera and point)", p);
            for (int pr : pbs[p].present) ch += (pr & 1) + (pr >> 1);
            nrec = (long long)pbs[p].pts.size();
            n_blocks += (int)pbs[p].cam0.size();
        } else {
            for (int j = 0; j < d.n_cams; ++j) ch += (cc[j] + BP - 1) / BP;
        }
        r.n_chunks = (int)ch;
        r.rec0 = n_recs; r.n_obs = d.n_obs;
        // consensus waves: consecutive points while their record groups fit
        // the 64 lanes
        {
            std::vector<int> nrec_pt(d.n_points, 0);
            if (k2)
                for (int pt : pbs[p].pts) ++nrec_pt[pt];
            else
                for (long long k = 0; k < d.n_obs; ++k) ++nrec_pt[d.obs_point[k]];
            r.cw0 = (int)out.cw_pt0.size();
            int lanes = CH;
            for (int i = 0; i < d.n_points; ++i) {
                const int g = cons_groups(nrec_pt[i]);
                if (lanes + g > CH) {
                    out.cw_pt0.push_back(n_pts + i);
                    lanes = 0;
                }
                lanes += g;
            }
            // whole workgroups of kConsWaves waves per problem (empty waves
            // start at the problem's end)
            while ((out.cw_pt0.size() - r.cw0) % kConsWaves) out.cw_pt0.push_back(n_pts + d.n_points);
            r.n_cw = (int)out.cw_pt0.size() - r.cw0;
        }
        out.ranges.push_back(r);
        n_cams += d.n_cams;
        n_pts += d.n_points;
        n_chunks += ch;
        n_recs += nrec;
    }
    const long long S = n_chunks * CH;
    if (S >= (1LL << 31) || n_recs >= (1LL << 31))
        return set_err(err, DBA_E_INVALID_ARG, "problem set too large (%lld slots)", S);
    out.n_slots = S;
    out.n_chunks = n_chunks;
    out.n_recs = n_recs;
    out.n_cams = n_cams;
    out.n_pts = n_pts;
    out.n_cw = (int)out.cw_pt0.size();
    out.cw_pt0.push_back(n_pts);
    out.n_blocks2 = k2 ? n_blocks : 0;

    out.uv.assign(2 * (size_t)S, R(0));
    out.pslot.assign(S, -1);
    out.ptid.assign(S, 0);
    out.orig.assign(S, 0);
    // per-observation camera copies; block local updates keep one per chunk
    const size_t SY = per_obs ? (size_t)S : 0;
    out.copy_y.assign(9 * SY, R(0));
    out.xrec.assign(3 * (size_t)n_recs, R(0));
    out.pt_off.assign(n_pts + 1, 0);
    out.chunk_cam.assign(n_chunks, 0);
    out.chunk_prob.assign(n_chunks, 0);
    out.cam_prob.assign(n_cams, 0);
    out.pt_prob.assign(n_pts, 0);
    out.cam_chunk0.assign(n_cams + 1, 0);
    out.cam_count.assign(n_cams, 0);
    out.cons_y.assign((size_t)n_cams * kConsY, 0.0);
    out.cons_x.assign(4 * (size_t)n_pts, 0.0);
    // two-camera blocks: chunk of each pair camera (or -1), record of each lane (or -1)
    out.blk_chunk.assign(k2 ? 2 * (size_t)n_blocks : 0, -1);
    out.blk_rec.assign(k2 ? (size_t)n_blocks * CH : 0, -1);
    out.blk_cam.assign(k2 ? 2 * (size_t)n_blocks : 0, -1);
    out.blk_prob.assign(k2 ? (size_t)n_blocks : 0, 0);
    out.blk_pt.assign(k2 ? (size_t)n_blocks * CH : 0, -1);
    int blk_base = 0;
    auto set_uv = [&](long long sl, const double *z) {
        out.uv[2 * sl] = (R)z[0];
        out.uv[2 * sl + 1] = (R)z[1];
    };
    auto set_x = [&](long long rec, const double *X) {
        for (int c = 0; c < 3; ++c) out.xrec[3 * rec + c] = (R)X[c];
    };

    for (int p = 0; p < np; ++p) {
        const dba_problem_desc &d = probs[p];
        const ProblemRange &r = out.ranges[p];
        const long long L = d.n_obs;
        // point-major records, stable in observation order (two-camera
        // blocks: a record per point copy, in block order within a point)
        std::vector<int> poff(d.n_points + 1, 0);
        if (k2)
            for (int pt : pbs[p].pts) ++poff[pt + 1];
        else
            for (long long k = 0; k < L; ++k) ++poff[d.obs_point[k] + 1];
        for (int i = 0; i < d.n_points; ++i) poff[i + 1] += poff[i];
        std::vector<int> fill(poff.begin(), poff.end() - 1);
        std::vector<int> rec_obs(k2 ? 0 : L);
        if (!k2)
            for (long long k = 0; k < L; ++k) rec_obs[fill[d.obs_point[k]]++] = (int)k;
        for (int i = 0; i <= d.n_points; ++i) out.pt_off[r.pt0 + i] = (int)(r.rec0 + poff[i]);
        for (int i = 0; i < d.n_points; ++i) {
            out.pt_prob[r.pt0 + i] = p;
            for (int c = 0; c < 3; ++c) out.cons_x[4 * (size_t)(r.pt0 + i) + c] = d.points[3 * i + c];
        }
        // camera-major slots, stable in record order
        std::vector<int> cc(d.n_cams, 0);
        for (long long k = 0; k < L; ++k) ++cc[d.obs_cam[k]];
        std::vector<long long> cslot(d.n_cams);
        std::vector<int> cseen(d.n_cams, 0);
        int chunk = r.chunk0;
        if (k2) {
            // chunks camera-major: camera j's chunks are its pair's blocks that it observes
            const PairBlocks &pb = pbs[p];
            const int nb = (int)pb.cam0.size();
            std::vector<int> brec(pb.pts.size());
            for (size_t t = 0; t < pb.pts.size(); ++t) brec[t] = (int)(r.rec0 + fill[pb.pts[t]]++);
            for (int b = 0; b < nb; ++b) {
                out.blk_prob[blk_base + b] = p;
                for (int l = 0; l < pb.npts[b]; ++l) {
                    const int t = pb.pts0[b] + l;
                    out.blk_rec[(size_t)(blk_base + b) * CH + l] = brec[t];
                    out.blk_pt[(size_t)(blk_base + b) * CH + l] = r.pt0 + pb.pts[t];
                    set_x(brec[t], d.points + 3LL * pb.pts[t]);
                }
            }
            int b0 = 0;
            for (int j = 0; j < d.n_cams; ++j) {
                const int J = r.cam0 + j, sc = j & 1;
                out.cam_prob[J] = p;
                out.cam_chunk0[J] = chunk;
                out.cam_count[J] = cc[j];
                for (int c = 0; c < 9; ++c) out.cons_y[(size_t)J * kConsY + c] = d.cams[9 * j + c];
                if (sc == 0) b0 = (int)(std::lower_bound(pb.cam0.begin(), pb.cam0.end(), j) - pb.cam0.begin());
                for (int b = b0; b < nb && pb.cam0[b] == j - sc; ++b) {
                    if (!(pb.present[b] >> sc & 1)) continue;
                    out.blk_chunk[2 * (size_t)(blk_base + b) + sc] = chunk;
                    out.blk_cam[2 * (size_t)(blk_base + b) + sc] = J;
                    out.chunk_cam[chunk] = J;
                    out.chunk_prob[chunk] = p;
                    for (int l = 0; l < pb.npts[b]; ++l) {
                        const int t = pb.pts0[b] + l;
                        const long long k = pb.obs[2 * (size_t)t + sc];
                        if (k < 0) continue;
                        const long long sl = (long long)chunk * CH + l;
                        out.pslot[sl] = brec[t];
                        out.ptid[sl] = r.pt0 + pb.pts[t];
                        out.orig[sl] = (int)k;
                        set_uv(sl, d.obs_uv + 2 * k);
                    }
                    ++chunk;
                }
            }
            blk_base += nb;
        } else {
            for (int j = 0; j < d.n_cams; ++j) {
                const int J = r.cam0 + j;
                out.cam_prob[J] = p;
                out.cam_chunk0[J] = chunk;
                out.cam_count[J] = cc[j];
                cslot[j] = (long long)chunk * CH;
                const int nch = (cc[j] + BP - 1) / BP;
                for (int q = 0; q < nch; ++q) {
                    out.chunk_cam[chunk + q] = J;
                    out.chunk_prob[chunk + q] = p;
                }
                chunk += nch;
                for (int c = 0; c < 9; ++c) out.cons_y[(size_t)J * kConsY + c] = d.cams[9 * j + c];
            }
            for (long long rr = 0; rr < L; ++rr) {
                const int k = rec_obs[rr];
                const int j = d.obs_cam[k], i = d.obs_point[k];
                const int q = cseen[j]++;
                const long long s = cslot[j] + (long long)(q / BP) * CH + q % BP;
                out.pslot[s] = (int)(r.rec0 + rr);
                out.ptid[s] = r.pt0 + i;
                out.orig[s] = k;
                set_uv(s, d.obs_uv + 2LL * k);
                if (per_obs)
                    for (int c = 0; c < 9; ++c) out.copy_y[(size_t)c * S + s] = (R)d.cams[9 * j + c];
                set_x(r.rec0 + rr, d.points + 3LL * i);
            }
        }
    }
    out.cam_chunk0[n_cams] = (int)n_chunks;
    // camera copy per chunk (block local updates), starting at the initial camera
    out.copy_yc.assign(9 * (size_t)n_chunks, R(0));
    for (long long c = 0; c < n_chunks; ++c)
        for (int i = 0; i < 9; ++i) out.copy_yc[9 * c + i] = (R)out.cons_y[(size_t)out.chunk_cam[c] * kConsY + i];
    return DBA_OK;
}

template int build_layout<float>(const LayoutOptions &, int, const dba_problem_desc *, Layout<float> *,
                                 std::string *);
template int build_layout<double>(const LayoutOptions &, int, const dba_problem_desc *, Layout<double> *,
                                  std::string *);

}  // namespace dba
