"""Algorithmic work of one ADMM iteration per observation, used to place
measured kernel times on the MI355X rooflines.

FLOPs count the arithmetic the local-solve algorithm performs (an FMA is 2,
every add/mul/compare-free arithmetic op is 1, each sqrt / rsqrt / rcp /
sin / cos / log is counted as 1); bytes count each piece of per-observation
state read or written once per iteration.
"""
from __future__ import annotations

# --- local solve (per observation) -----------------------------------------
# projection with Jacobian: Rodrigues coefficients 25, transform 36, perspective
# + distortion 14, d pi / d P 24, q 16, two Jacobian rows 2 x 70
PROJ_JAC = 25 + 36 + 14 + 24 + 16 + 140
# projection only (trial point): coefficients 16, transform 36, perspective 14
PROJ = 16 + 36 + 14
# residual, loss weight and resolution of F
RESID = 5 + 6 + 6
# normal equations: for each row 12 (gradient, scale), 78 packed entries x 3,
# diagonal + damping 24
NORMAL = 12 * 10 + 78 * 3 + 24
# packed 12x12 Cholesky: sum_j 2j + sum_j (11-j)(2j+1) + 12 rsqrt
CHOL = 132 + 506 + 12
# forward + backward substitution
SOLVE = 2 * 144
# trial point, predicted decrease, objective at the trial (projection,
# residual, loss, 12-term penalty), acceptance
TRIAL = 12 + 60 + 3 + PROJ + 10 + 36 + 15
LM_STEP = PROJ_JAC + RESID + NORMAL + CHOL + SOLVE + TRIAL
# per solve: initial objective, deferred dual update (12 x 3), v (12),
# chunk sums (19 values, 6 butterfly adds each, plus forming them 40)
PER_SOLVE = (PROJ + 10 + 36) + 36 + 12 + 19 * 6 + 40


def local_flops_per_obs(lm_steps: int = 5) -> int:
    return PER_SOLVE + lm_steps * LM_STEP


# --- bytes per observation per iteration --------------------------------------
def bytes_per_obs(fp32: bool = True) -> dict:
    r = 4 if fp32 else 8
    local = (2 * r          # uv
             + 4 + 4        # point record index, point id
             + 2 * 9 * r    # camera-side copy read + write
             + 2 * 9 * 8    # camera-side scaled dual read + write
             + 2 * 4 * r    # point-side copy record read + write (4-wide)
             + 2 * 4 * 8)   # point-side dual record read + write (4-wide)
    consensus = 4 * r + 4 * 8   # point records read once more
    minimal = 2 * r + 8 + 2 * 12 * r + 2 * 12 * 8   # obs + indices + copies r/w + duals r/w
    return dict(local=local, consensus=consensus, total=local + consensus, minimal=minimal)


if __name__ == "__main__":
    print("LM step flops", LM_STEP, "per obs (5 steps)", local_flops_per_obs(5))
    print("bytes fp32", bytes_per_obs(True), "fp64", bytes_per_obs(False))
