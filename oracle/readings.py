"""Readings taken where the paper is silent, ambiguous or garbled.

Each entry: (id, passage, reading). The oracle and the GPU library both follow
these; they are repeated in the design notes.
"""

READINGS = [
    ("R1", "Sec. II-B, 'sufficient texture'",
     "Central-difference gradient magnitude of the keyframe image >= 6 grey levels "
     "(0-255 scale), compared as gx^2 + gy^2 >= 36 so the decision is exact; a 2-pixel "
     "border is excluded. Computed once per keyframe."),
    ("R2", "Sec. II-B, 'five equally spaced points'",
     "LINE5: five points at 1-pixel spacing along the epipolar line through the pixel in "
     "the keyframe and along the epipolar line in the new frame. SQ5X5: a 5x5 square patch "
     "with a translation-only warp (the 5x5 patch of the workload descriptions)."),
    ("R3", "Sec. II-B, interval d +- 2 sigma",
     "The filter lives in inverse depth rho; the search interval is rho +- 2 sqrt(v), "
     "clamped to [1/d_far, 1/d_near] (agrees with d +- 2 sigma_d to first order)."),
    ("R4", "Sec. II-B, 'the entire epipolar line'",
     "The inverse-depth range [1/d_far, 1/d_near] with d_near = 0.4 m, d_far = 10 m."),
    ("R5", "Sec. II-B, 1-pixel steps",
     "Always N_s samples, centred on the interval's image segment, step "
     "h = max(1 px, L/(N_s-1)). Samples beyond the interval but inside the global "
     "inverse-depth range are valid."),
    ("R6", "Sec. II-B, interpolation between two steps",
     "Endpoints: the SSD minimum k* and its lower-SSD valid neighbour (tie -> k*-1). "
     "lambda* minimises |e_k* + lambda de|^2, clipped to [0, 1]; depth is interpolated "
     "linearly in depth."),
    ("R7", "Sec. II-B, eq. (semi)",
     "Photometric noise sigma_I = 1 grey level: sigma_d^2 = sigma_I^2 dd^2 / (de^T de)."),
    ("R8", "Sec. II, filter of the cited semi-dense method",
     "Gaussian product in inverse depth, first-order conversion v_o = sigma_d^2 / d^4, "
     "no process noise, no outlier counters; a failed search leaves the state unchanged."),
    ("R9", "Sec. II-B, conversion to log space",
     "z = ln d_semi = -ln rho, R = v / rho^2 (first order), floored at R_floor = 1e-6."),
    ("R10", "Sec. II-C, gradient terms at the border",
     "x-edges exist for u < W-1, y-edges for v < H-1; the prediction in the last "
     "column / row is unused."),
    ("R12", "Sec. II-C, Huber loss",
     "Huber on whitened residuals r/sigma with delta = 1.345: H(r) = r^2 for |r| <= delta, "
     "2 delta |r| - delta^2 otherwise; IRLS weight min(1, delta/|r|); delta = inf gives "
     "plain weighted least squares."),
    ("R13", "Sec. II-C, alternating depth and scale",
     "Each Gauss-Newton iteration: IRLS weights at (x, tau) -> solve for x with tau fixed "
     "-> semi weights at the new x -> closed-form tau = sum w (x - z) / sum w. Depth "
     "first; tau unchanged when no semi-dense measurement exists."),
    ("R14", "Sec. II-C, inner solver",
     "Oracle: direct sparse solve, or Jacobi PCG with the same warm start and iteration "
     "count as the GPU (iteration-matched). GPU: Jacobi PCG."),
    ("R15", "Workload '20 CG iterations per frame'",
     "10 Gauss-Newton iterations (Sec. II-C) x 20 PCG iterations each."),
    ("R16", "Sec. II-C, 'the set of log-depth values'",
     "The unknown per pixel is x = ln d; the scale is solved as tau = ln s."),
    ("R19", "Sec. II-B, back-projection",
     "z-depth: rho(x, d) = d K^-1 (u, v, 1); integer coordinates are pixel centres."),
]
