"""Algorithmic work of one ADMM iteration per observation, used to place
measured kernel times on the MI355X rooflines.

FLOPs count the arithmetic the local-solve algorithm performs (an FMA is 2,
every add/mul/compare-free arithmetic op is 1, each sqrt / rsqrt / rcp /
sin / cos / log is counted as 1); bytes count each piece of per-observation
state read or written once per iteration.
"""
from __future__ import annotations

# --- local solve (per observation) -----------------------------------------
# projection core (also the trial evaluation): Rodrigues coefficients with
# their derivatives 25, transform 36, perspective + distortion 14
PROJ = 25 + 36 + 14
# Jacobian rows from the cached projection: d pi / d P 24, q 16, 2 rows x 70
JAC = 24 + 16 + 140
# residual, loss weight, resolution of F
RESID = 5 + 6 + 6
# negative gradient (7), diag(H) (5), Marquardt diagonal (2), per parameter
GRAD = 12 * 14
# LDL^T of D + c (J0 J0^T + J1 J1^T): rank-one update 1 (9 per row),
# L1^-1 J1 and rank-one update 2 (12 per row)
FACTOR = 12 * 9 + 12 * 12
# L1^-1, L2^-1, D2^-1, L2^-T, L1^-T
SOLVE = 4 * 48 + 12
# trial point 12, predicted decrease 63, objective at the trial (projection,
# residual 5, loss 5, 12-term penalty 36, total 2), acceptance 30
TRIAL = 12 + 63 + PROJ + 48 + 30
LM_STEP = JAC + RESID + GRAD + FACTOR + SOLVE + TRIAL
# per solve: initial projection and objective, deferred dual update (12 x 3),
# v (12), chunk sums (19 values, 6 butterfly adds each, plus forming them 40)
PER_SOLVE = (PROJ + 48) + 36 + 12 + 19 * 6 + 40


def local_flops_per_obs(lm_steps: int = 5, camera: str = "angle_axis") -> int:
    if camera == "euler":
        return PER_SOLVE_E + lm_steps * LM_STEP_E
    return PER_SOLVE + lm_steps * LM_STEP


# --- the Euler camera of Eq. (1): 6 camera + 3 point unknowns -----------------
# the algorithmic work of the paper's 9-unknown local problem (the kernel also
# carries the 3 unused camera slots through its 12-wide solve; not counted).
# projection: three sincos (2 each), X1 = R1 X, X2 = R2 X1, Q = R3 X2 (6 x 3),
# translation 3, perspective and focal length 5
PROJ_E = 6 + 18 + 3 + 5
# Jacobian rows: A 3, per row c = a R3 (6), b = c R2 (6), three angle columns
# (9), point columns (6)
JAC_E = 3 + 2 * 27
GRAD_9 = 9 * 14
FACTOR_9 = 9 * 9 + 9 * 12
SOLVE_9 = 4 * 36 + 9
# trial point 9, predicted decrease 47, objective at the trial (projection,
# residual 5, loss 5, 9-term penalty 27, total 2), acceptance 30
TRIAL_9 = 9 + 47 + PROJ_E + 39 + 30
LM_STEP_E = JAC_E + RESID + GRAD_9 + FACTOR_9 + SOLVE_9 + TRIAL_9
PER_SOLVE_E = (PROJ_E + 39) + 27 + 9 + 19 * 6 + 40


# --- block local updates (one camera copy per 64 observations) -------------------
# per observation and LM step: projection, Jacobian and residual as above;
# the camera-camera (45), camera-point (27), point-point (6) blocks and both
# gradients 366; the damped 3x3 point block inverted 40; its Schur
# contribution to the 9x9 camera system and right-hand side 459; the
# all-reduce's additions 63; the point step 72; predicted decrease 15; trial
# projection and objective 95.  The 9x9 LDL^T and its solves (420) are once
# per block of 64 observations.
BLOCK_LM_STEP = JAC + RESID + 366 + 40 + 459 + 63 + 72 + 15 + PROJ + 20 + 420 // 64
BLOCK_PER_SOLVE = PROJ + 20 + 3 * 3 + 9 * 3 // 64


# --- two-camera blocks (a copy per block point, up to two observations each) ---
# per observation and LM step: projection, Jacobian and residual; its part of
# the point block and gradient 36; B V for its two rows 30; r 16; its camera
# rows' right-hand side, gradient and diagonal values 108; its part of W^T dy
# 48; trial projection and objective 95.  Per point copy: the damped 3x3 block
# inverted 40; M for the three camera pairs 108; Q 216; the 171 reduced-system
# values 684; the point step and predicted decrease 45.  Per block of 64
# copies: the 18x18 LDL^T (1 944) and its solves (684), and the all-reduce's
# additions (226 per copy).
BLOCK2_OBS_STEP = JAC + RESID + 36 + 30 + 16 + 108 + 48 + PROJ + 20
BLOCK2_COPY_STEP = 40 + 108 + 216 + 684 + 45 + 226 + (1944 + 684) // 64


def block2_flops_per_obs(lm_steps: int = 5, obs_per_copy: float = 1.7) -> int:
    return int(round((BLOCK_PER_SOLVE + lm_steps * (BLOCK2_OBS_STEP + BLOCK2_COPY_STEP / obs_per_copy))))


def block_flops_per_obs(lm_steps: int = 5) -> int:
    return BLOCK_PER_SOLVE + lm_steps * BLOCK_LM_STEP


# --- bytes per observation per iteration --------------------------------------
def bytes_per_obs(fp32: bool = True) -> dict:
    r = 4 if fp32 else 8
    local = (2 * r          # uv
             + 4 + 4        # point record index, point id
             + 2 * 9 * r    # camera-side copy read + write
             + 2 * 9 * 8    # camera-side scaled dual read + write
             + 2 * 3 * r    # point-side copy record read + write
             + 2 * 3 * 8)   # point-side dual record read + write
    consensus = 3 * r + 3 * 8   # point records read once more
    minimal = 2 * r + 8 + 2 * 12 * r + 2 * 12 * 8   # obs + indices + copies r/w + duals r/w
    return dict(local=local, consensus=consensus, total=local + consensus, minimal=minimal)


def obs_per_block(obs_cams, block_points: int = 64) -> float:
    """Mean observations per block when each camera's observations are cut
    into consecutive blocks of block_points (one-camera blocks)."""
    import numpy as np
    n_obs = n_blocks = 0
    for oc in obs_cams:
        cnt = np.bincount(np.asarray(oc))
        n_obs += int(cnt.sum())
        n_blocks += int(((cnt + block_points - 1) // block_points).sum())
    return n_obs / max(n_blocks, 1)


def block_bytes_per_obs(fp32: bool = True, obs_per_block: float = 64.0) -> float:
    """One-camera blocks: per observation its pixel, indexes, point copy and
    point dual; per block one camera copy and dual, read and written."""
    r = 4 if fp32 else 8
    return 2 * r + 8 + 2 * 3 * r + 2 * 3 * 8 + (2 * 9 * r + 2 * 9 * 8) / obs_per_block


def block2_bytes_per_obs(fp32: bool = True, obs_per_copy: float = 1.7) -> float:
    """Two-camera blocks: per observation its pixel and indexes; per point
    copy its copy and dual, read and written (the block cameras' copies, one
    per pair and block, are negligible)."""
    r = 4 if fp32 else 8
    return 2 * r + 8 + (2 * 3 * r + 2 * 3 * 8) / obs_per_copy


if __name__ == "__main__":
    print("LM step flops", LM_STEP, "per obs (5 steps)", local_flops_per_obs(5))
    print("Euler camera: LM step flops", LM_STEP_E, "per obs (5 steps)", local_flops_per_obs(5, "euler"))
    print("bytes fp32", bytes_per_obs(True), "fp64", bytes_per_obs(False))
    print("block LM step flops", BLOCK_LM_STEP, "per obs (5 steps)", block_flops_per_obs(5))
