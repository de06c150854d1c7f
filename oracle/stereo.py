"""Semi-dense estimation (Sec. II-B): epipolar search, interpolation, variance, filter.

Plain and slow on purpose: numpy over the searched pixels, a Python loop over
the epipolar samples and the pattern points, every sample evaluated (brute
force), nothing blocked or fused. ``dtype`` selects the precision of every
per-pixel operation (float64 by default; float32 to take integer decisions
such as the SSD argmin in the precision a float32 kernel uses).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import epipolar_constants, project_through

# skip reasons of one pixel's search (0 = measurement produced)
UPDATED = 0
EMPTY_INTERVAL = 1
BEHIND_CAMERA = 2
DEGENERATE_LINE = 3
NO_VALID_SAMPLE = 4
NO_NEIGHBOUR = 5
FLAT_ERROR = 6


@dataclass
class StereoParams:
    n_samples: int = 32          # N_s equally spaced samples per pixel (R5)
    pattern: str = "line5"       # "line5" (Sec. II-B, five points) or "sq5x5" (R2)
    d_near: float = 0.4          # R4
    d_far: float = 10.0          # R4
    grad_gate: float = 6.0       # R1
    sigma_photo: float = 1.0     # R7
    border: int = 2              # pattern half-width


def texture_mask(image0: np.ndarray, grad_gate: float = 6.0, border: int = 2) -> np.ndarray:
    """Pixels with 'sufficient texture' (Sec. II-B, reading R1).

    Central differences of the uint8 keyframe image; |grad|^2 >= gate^2 (exact
    for integer images); a border of ``border`` pixels is never searched.
    """
    I = np.asarray(image0, dtype=np.float64)
    H, W = I.shape
    gx = np.zeros_like(I)
    gy = np.zeros_like(I)
    gx[:, 1:-1] = (I[:, 2:] - I[:, :-2]) / 2.0
    gy[1:-1, :] = (I[2:, :] - I[:-2, :]) / 2.0
    mask = gx * gx + gy * gy >= grad_gate * grad_gate
    if border > 0:
        mask[:border, :] = False
        mask[-border:, :] = False
        mask[:, :border] = False
        mask[:, -border:] = False
    return mask


def bilinear(img: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Bilinear intensity at (u, v) for 0 <= u <= W-1, 0 <= v <= H-1.

    u0 = min(floor(u), W-2), f = u - u0 (likewise v); the four taps are weighted
    (1-f)(1-g), f(1-g), (1-f)g, fg.
    """
    H, W = img.shape
    fu = np.minimum(np.floor(u), W - 2)
    fv = np.minimum(np.floor(v), H - 2)
    f = u - fu
    g = v - fv
    iu = fu.astype(np.int64)
    iv = fv.astype(np.int64)
    I00 = img[iv, iu]
    I10 = img[iv, iu + 1]
    I01 = img[iv + 1, iu]
    I11 = img[iv + 1, iu + 1]
    one = img.dtype.type(1)
    return (one - f) * (one - g) * I00 + f * (one - g) * I10 + (one - f) * g * I01 + f * g * I11


def _inside(u, v, W, H):
    return (u >= 0) & (u <= W - 1) & (v >= 0) & (v <= H - 1)


@dataclass
class SearchResult:
    """Per searched pixel (row-major order of the texture mask)."""
    pix: np.ndarray        # flat pixel indices searched
    status: np.ndarray     # UPDATED or a skip reason
    ssd: np.ndarray        # (npix, N_s) SSD of every sample, +inf where invalid
    rho_k: np.ndarray      # (npix, N_s) inverse depth of every sample
    k_best: np.ndarray     # k*, -1 if none
    k_nbr: np.ndarray      # n*, -1 if none
    lam: np.ndarray        # lambda*
    d_star: np.ndarray     # interpolated depth
    var_d: np.ndarray      # sigma_d^2 of eq. (semi)
    rho_obs: np.ndarray    # 1 / d*
    var_obs: np.ndarray    # sigma_d^2 / d*^4
    tap_margin: np.ndarray = None    # (npix, N_s) px from the sample's nearest tap to the image edge (< 0: outside)
    range_margin: np.ndarray = None  # (npix, N_s) min(rho_k - rho_min, rho_max - rho_k) / rho_k (< 0: outside)


def _pattern(I0f, u, v, l0x, l0y, pattern, dt):
    """Keyframe pattern values and the matching image-1 offsets (R2)."""
    if pattern == "line5":
        js = [dt.type(j) for j in (-2, -1, 0, 1, 2)]
        vals = [bilinear(I0f, u + j * l0x, v + j * l0y) for j in js]
        return vals, js
    if pattern == "sq5x5":
        iu = u.astype(np.int64)
        iv = v.astype(np.int64)
        vals, offs = [], []
        for n in (-2, -1, 0, 1, 2):
            for m in (-2, -1, 0, 1, 2):
                vals.append(I0f[iv + n, iu + m])
                offs.append((dt.type(m), dt.type(n)))
        return vals, offs
    raise ValueError(pattern)


def _taps(pattern, offs, pkx, pky, lx, ly):
    """Image-1 points of one sample: p_k + j l1 (LINE5) or p_k + (m, n) (SQ5X5)."""
    if pattern == "line5":
        return [(pkx + j * lx, pky + j * ly) for j in offs]
    return [(pkx + m, pky + n) for (m, n) in offs]


def epipolar_search(I0, I1, K, T_wc0, T_wc1, rho, var, valid, mask,
                    params: StereoParams, dtype=np.float64) -> SearchResult:
    """One frame's search for every textured keyframe pixel (Sec. II-B).

    rho, var, valid: the current inverse-depth filter state (H x W); a valid
    pixel is searched over rho +- 2 sqrt(var), others over the whole range.
    """
    dt = np.dtype(dtype)
    I0 = np.asarray(I0)
    H, W = I0.shape
    Hd, bd, ed = epipolar_constants(K, T_wc0, T_wc1)
    Hinf = Hd.astype(dt)
    b = bd.astype(dt)
    e0 = ed.astype(dt)
    I0f = I0.astype(dt)
    I1f = np.asarray(I1).astype(dt)
    NS = int(params.n_samples)
    pix = np.flatnonzero(np.asarray(mask).ravel())
    n = pix.size
    u = (pix % W).astype(dt)
    v = (pix // W).astype(dt)
    rmin = dt.type(1.0 / params.d_far)
    rmax = dt.type(1.0 / params.d_near)
    two = dt.type(2)

    status = np.full(n, UPDATED, dtype=np.int32)

    # interval in inverse depth (R3, R4)
    rs = np.asarray(rho).ravel()[pix].astype(dt)
    vs = np.asarray(var).ravel()[pix].astype(dt)
    has = np.asarray(valid).ravel()[pix].astype(bool)
    sd = np.sqrt(np.where(has, vs, dt.type(0)))
    lo = np.where(has, np.maximum(rs - two * sd, rmin), rmin)
    hi = np.where(has, np.minimum(rs + two * sd, rmax), rmax)
    status[~(hi > lo)] = EMPTY_INTERVAL

    # image-1 segment of the interval
    plx, ply, dlo = project_through(Hinf, b, u, v, lo)
    phx, phy, dhi = project_through(Hinf, b, u, v, hi)
    behind = ~((dlo > 0) & (dhi > 0))
    status[(status == UPDATED) & behind] = BEHIND_CAMERA
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        dx = phx - plx
        dy = phy - ply
        L = np.sqrt(dx * dx + dy * dy)
        lx = dx / L
        ly = dy / L
    short = ~(np.isfinite(L) & (L >= dt.type(1e-6)))
    status[(status == UPDATED) & short] = DEGENERATE_LINE
    h = np.maximum(dt.type(1), L / dt.type(NS - 1))
    cx = (plx + phx) / two
    cy = (ply + phy) / two
    use_x = np.abs(lx) >= np.abs(ly)
    A0 = Hinf[0, 0] * u + Hinf[0, 1] * v + Hinf[0, 2]
    A1 = Hinf[1, 0] * u + Hinf[1, 1] * v + Hinf[1, 2]
    A2 = Hinf[2, 0] * u + Hinf[2, 1] * v + Hinf[2, 2]

    # keyframe epipolar direction for LINE5 (through the epipole e0 = K c1)
    l0x = np.zeros(n, dtype=dt)
    l0y = np.zeros(n, dtype=dt)
    if params.pattern == "line5":
        with np.errstate(invalid="ignore", divide="ignore"):
            ddx = e0[2] * u - e0[0]
            ddy = e0[2] * v - e0[1]
            n0 = np.sqrt(ddx * ddx + ddy * ddy)
            l0x = ddx / n0
            l0y = ddy / n0
            rc = (lo + hi) / two
            q0x, q0y, _ = project_through(Hinf, b, u, v, rc)
            q1x, q1y, _ = project_through(Hinf, b, u + l0x, v + l0y, rc)
            flip = (q1x - q0x) * lx + (q1y - q0y) * ly < 0
        l0x = np.where(flip, -l0x, l0x)
        l0y = np.where(flip, -l0y, l0y)
        bad0 = ~(np.isfinite(l0x) & np.isfinite(l0y) & (n0 > 0))
        status[(status == UPDATED) & bad0] = DEGENERATE_LINE
        l0x = np.where(bad0, dt.type(0), l0x)
        l0y = np.where(bad0, dt.type(0), l0y)

    live = status == UPDATED
    # keep arithmetic finite on dead pixels
    lx = np.where(live, lx, dt.type(1))
    ly = np.where(live, ly, dt.type(0))
    h = np.where(live, h, dt.type(1))
    cx = np.where(live, cx, u)
    cy = np.where(live, cy, v)

    pat0, offs = _pattern(I0f, u, v, l0x, l0y, params.pattern, dt)
    P = len(pat0)

    ssd = np.full((n, NS), np.inf, dtype=dt)
    rho_k = np.zeros((n, NS), dtype=dt)
    tap_margin = np.full((n, NS), -np.inf)
    range_margin = np.full((n, NS), -np.inf)
    half = dt.type((NS - 1) / 2.0)
    for k in range(NS):
        off = dt.type(k) - half
        pkx = cx + off * h * lx
        pky = cy + off * h * ly
        pm = np.where(use_x, pkx, pky)
        Am = np.where(use_x, A0, A1)
        bm = np.where(use_x, b[0], b[1])
        with np.errstate(invalid="ignore", divide="ignore"):
            rk = (pm * A2 - Am) / (bm - pm * b[2])
        ok = live & np.isfinite(rk) & (rk >= rmin) & (rk <= rmax)
        taps = _taps(params.pattern, offs, pkx, pky, lx, ly)
        for (tu, tv) in taps:
            ok &= _inside(tu, tv, W, H)
        # how far each validity test is from its boundary (reported, not used)
        tm = np.full(n, np.inf)
        for (tu, tv) in taps:
            tm = np.minimum(tm, np.minimum(np.minimum(tu, W - 1 - tu), np.minimum(tv, H - 1 - tv)))
        tap_margin[:, k] = np.where(live, tm, -np.inf)
        with np.errstate(invalid="ignore", divide="ignore"):
            rm = np.minimum(rk - rmin, rmax - rk) / rk
        range_margin[:, k] = np.where(live & np.isfinite(rk), rm, -np.inf)
        s = np.zeros(n, dtype=dt)
        for j, (tu, tv) in enumerate(taps):
            cu = np.clip(np.where(ok, tu, dt.type(0)), 0, W - 1).astype(dt)
            cv = np.clip(np.where(ok, tv, dt.type(0)), 0, H - 1).astype(dt)
            e = bilinear(I1f, cu, cv) - pat0[j]
            s = s + e * e
        ssd[:, k] = np.where(ok, s, dt.type(np.inf))
        rho_k[:, k] = np.where(np.isfinite(rk), rk, dt.type(0))

    anyv = np.isfinite(ssd).any(axis=1)
    status[(status == UPDATED) & ~anyv] = NO_VALID_SAMPLE
    rows = np.arange(n)
    kb = np.argmin(ssd, axis=1)                    # first minimum: ties -> smallest k
    km = kb - 1
    kp = kb + 1
    s_m = np.where(km >= 0, ssd[rows, np.clip(km, 0, NS - 1)], np.inf)
    s_p = np.where(kp < NS, ssd[rows, np.clip(kp, 0, NS - 1)], np.inf)
    nb = np.where(s_m <= s_p, km, kp)              # tie -> k* - 1
    has_nb = np.isfinite(s_m) | np.isfinite(s_p)
    status[(status == UPDATED) & ~has_nb] = NO_NEIGHBOUR
    nb = np.clip(nb, 0, NS - 1)

    def residuals(kidx):
        off = kidx.astype(dt) - half
        pkx = cx + off * h * lx
        pky = cy + off * h * ly
        taps = _taps(params.pattern, offs, pkx, pky, lx, ly)
        out = np.empty((n, P), dtype=dt)
        for j, (tu, tv) in enumerate(taps):
            cu = np.clip(tu, 0, W - 1).astype(dt)
            cv = np.clip(tv, 0, H - 1).astype(dt)
            out[:, j] = bilinear(I1f, cu, cv) - pat0[j]
        return out

    ok_rows = status == UPDATED
    ek = residuals(kb)
    en = residuals(nb)
    de = en - ek                                   # difference at the two endpoints
    dd = np.sum(de * de, axis=1)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        lam = np.clip(-np.sum(ek * de, axis=1) / dd, dt.type(0), dt.type(1))
        d_a = dt.type(1) / rho_k[rows, kb]
        d_b = dt.type(1) / rho_k[rows, nb]
        ddep = d_b - d_a
        d_star = d_a + lam * ddep
        # eq. (semi): J = de / dd_semi, sigma^2 = (J^T J)^-1, times sigma_I^2 (R7)
        var_d = dt.type(params.sigma_photo) ** 2 * ddep * ddep / dd
        rho_o = dt.type(1) / d_star
        d2 = d_star * d_star
        var_o = var_d / (d2 * d2)
    good = ok_rows & (dd > 0) & np.isfinite(var_d) & (var_d > 0) & np.isfinite(d_star) & (d_star > 0) \
        & np.isfinite(var_o) & (var_o > 0)
    status[ok_rows & ~good] = FLAT_ERROR
    fin = status == UPDATED
    kb_out = np.where(anyv & (status != EMPTY_INTERVAL) & (status != BEHIND_CAMERA)
                      & (status != DEGENERATE_LINE), kb, -1)
    nb_out = np.where(fin, nb, -1)
    return SearchResult(pix, status, ssd, rho_k, kb_out, nb_out,
                        np.where(fin, lam, 0), np.where(fin, d_star, 0), np.where(fin, var_d, 0),
                        np.where(fin, rho_o, 0), np.where(fin, var_o, 0), tap_margin, range_margin)


def filter_update(rho, var, valid, pix, rho_obs, var_obs):
    """Inverse-depth Gaussian filter (reading R8): product of the prior and the observation.

    First observation: (rho, var) := (rho_o, var_o). Otherwise
    rho := (var_o rho + var rho_o) / (var + var_o), var := var var_o / (var + var_o).
    Returns new (rho, var, valid) arrays (H x W); inputs are not modified.
    """
    shape = np.shape(rho)
    r = np.array(rho, dtype=np.result_type(rho, rho_obs)).ravel()
    v = np.array(var, dtype=r.dtype).ravel()
    ok = np.array(valid, dtype=bool).ravel()
    rp = r[pix]
    vp = v[pix]
    op = ok[pix]
    fused_r = (var_obs * rp + vp * rho_obs) / (vp + var_obs)
    fused_v = vp * var_obs / (vp + var_obs)
    r[pix] = np.where(op, fused_r, rho_obs)
    v[pix] = np.where(op, fused_v, var_obs)
    ok[pix] = True
    return r.reshape(shape), v.reshape(shape), ok.reshape(shape)


def stereo_update(I0, I1, K, T_wc0, T_wc1, rho, var, valid, mask, params: StereoParams,
                  dtype=np.float64):
    """Search + filter for one new frame; returns (rho, var, valid, SearchResult)."""
    res = epipolar_search(I0, I1, K, T_wc0, T_wc1, rho, var, valid, mask, params, dtype)
    upd = res.status == UPDATED
    r, v, ok = filter_update(np.asarray(rho, dtype=np.dtype(dtype)), np.asarray(var, dtype=np.dtype(dtype)),
                             valid, res.pix[upd], res.rho_obs[upd], res.var_obs[upd])
    return r, v, ok, res


def log_measurements(rho, var, valid, r_floor: float = 1e-6):
    """Semi-dense estimates in log space (Sec. II-B last step, reading R9).

    z = ln d_semi = -ln rho and R = max(var / rho^2, R_floor) on valid pixels;
    z = 0 and R = +inf elsewhere.
    """
    ok = np.asarray(valid, dtype=bool)
    r = np.where(ok, rho, 1.0)
    z = np.where(ok, -np.log(r), 0.0)
    R = np.where(ok, np.maximum(np.asarray(var) / (r * r), r_floor), np.inf)
    return z, R, ok
