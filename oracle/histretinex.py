"""FP64 reference of the HistRetinex pipeline (Zhao et al., arXiv 2510.21100).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark; never by the GPU library.  It is deliberately slow
and literal: the l x l count, location, class and weight matrices of Sec. III-A
and III-B are materialised, every sum is a plain numpy reduction, and every
floating-point quantity is float64.

Notation follows the paper: S is the HSV value channel of the image (Sec. II),
l the number of levels, N the number of pixels.  Histograms of the
illumination L and reflectance R are carried in probability units (count / N);
the paper's count histograms are N times these.  Rows of every l x l matrix are
indexed by the illumination level a, columns by the reflectance level b.

Readings of passages the paper leaves open (each is also listed in the design
notes):
  * the gradient image is the forward-difference L1 magnitude
    |S(x+1,y)-S(x,y)| + |S(x,y+1)-S(x,y)| with a replicated last column / row,
    binned into 2l-1 raw levels and then rescaled so that its largest occupied
    raw level lands on level l-1 (Alg. 1, initialisation);
  * the location histogram H_B of any component is the vector of level
    positions k/(l-1); the "/N" printed in Eq. (7) and the second "/N" of
    Eq. (8) are dropped (otherwise every product falls into class 0);
  * index(.) and index_1(.) of Eqs. (10) and (19) are the arg-min over levels,
    ties to the smaller level;
  * Eqs. (12)-(13) multiply by K_ij: these are the stationarity conditions of
    Eq. (10) with K frozen, which is how the paper says it derived them;
  * K is 0 where its class total is 0; the initial illumination histogram is
    the image histogram; the updates run in the order of Alg. 1 (R by Eq. 13,
    then L by Eq. 12 with the new unnormalised R, then the normalisations of
    Eqs. 15 and 14, then K by Eq. 11);
  * the stopping rule of Alg. 1 is garbled; it is read as: stop after pass
    t when t = T (the maximum), or earlier when the squared Euclidean norms
    of the changes of both normalised histograms in that pass, in
    probability units, are at most eps; eps <= 0 runs exactly T passes;
  * the histogram matching back to pixels maps level v to the smallest target
    level whose cumulative target mass reaches the mid-rank source CDF at v,
    and only the value channel is replaced (hue and saturation kept), which
    for RGB is a per-pixel scaling of all channels by LUT[V]/V with
    round-half-up.
"""

from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np


#: gradient operators for H_C(grad S) (the paper does not define the operator)
GRAD_OPERATORS = ("fwd_l1", "fwd_l2", "sobel_l1")
#: how the raw gradient levels are put onto the l image levels
GRAD_RESCALES = ("max", "clip")
#: readings of Eqs. (12)-(13): multiply by K (stationarity of Eq. 10) or the
#: printed division by K
UPDATES = ("mul", "div")
#: initial illumination histogram: the image histogram, or uniform over all levels
INIT_L = ("image", "uniform")


@dataclass(frozen=True)
class Params:
    """Method parameters: bins l, iterations T (the maximum of Alg. 1), prior
    weights alpha, beta of Eq. (10), the illumination gamma of Eq. (17) and
    the error threshold eps of Alg. 1 (<= 0: exactly T passes).  The last
    four fields switch between readings of passages the paper leaves open
    (the defaults are the readings the pipeline is built on): the gradient
    operator and the rescaling of its histogram, the form of Eqs. (12)-(13),
    and the initial illumination histogram."""

    bins: int = 256
    iters: int = 50
    alpha: float = 0.01
    beta: float = 0.01
    gamma: float = 2.2
    eps: float = 0.0
    grad_op: str = "fwd_l1"
    grad_rescale: str = "max"
    update: str = "mul"
    init_l: str = "image"

    def __post_init__(self):
        if self.grad_op not in GRAD_OPERATORS:
            raise ValueError(f"grad_op must be one of {GRAD_OPERATORS}")
        if self.grad_rescale not in GRAD_RESCALES:
            raise ValueError(f"grad_rescale must be one of {GRAD_RESCALES}")
        if self.update not in UPDATES:
            raise ValueError(f"update must be one of {UPDATES}")
        if self.init_l not in INIT_L:
            raise ValueError(f"init_l must be one of {INIT_L}")


# --------------------------------------------------------------------------
# Pixel front end and histograms (Sec. II; Eq. 3; Alg. 1 initialisation)
# --------------------------------------------------------------------------

def value_channel(img: np.ndarray) -> np.ndarray:
    """HSV value channel: V = max(R, G, B) per pixel (Sec. II, notation)."""
    if img.ndim != 3 or img.shape[2] != 3:
        raise ValueError("expected an H x W x 3 image")
    return img.max(axis=2).astype(np.int64)


def count_histogram(values: np.ndarray, levels: int) -> np.ndarray:
    """H_C of Eq. (3): n_i = number of entries equal to level i."""
    v = np.asarray(values, dtype=np.int64).ravel()
    if v.size and (v.min() < 0 or v.max() >= levels):
        raise ValueError("value outside [0, levels)")
    return np.bincount(v, minlength=levels).astype(np.int64)


def _round_sqrt(q: np.ndarray) -> np.ndarray:
    """round-half-up(sqrt(q)) of non-negative integers, exactly: r = isqrt(q),
    plus one when q - r^2 > r (sqrt(q) >= r + 1/2 iff q >= r^2 + r + 1/4)."""
    q = np.asarray(q, dtype=np.int64)
    r = np.floor(np.sqrt(q.astype(np.float64))).astype(np.int64)
    r -= (r * r > q)          # isqrt: correct the float estimate downwards
    r += ((r + 1) * (r + 1) <= q)  # and upwards
    return r + (q - r * r > r)


def gradient_magnitude(V: np.ndarray, operator: str = "fwd_l1") -> np.ndarray:
    """Gradient image of the value channel (Alg. 1 initialisation; the operator
    is not given in the paper), integer levels in [0, 2(l-1)]:

      fwd_l1   forward differences, |dx| + |dy|, the last column and row
               replicated so their missing difference is 0 (the default);
      fwd_l2   the same differences, Euclidean magnitude sqrt(dx^2 + dy^2)
               rounded half up;
      sobel_l1 the 3x3 Sobel derivatives gx, gy on the image with its border
               replicated, (|gx| + |gy|) / 4 rounded half up (the Sobel
               weights sum to 4, so a step of height h gives h).
    """
    V = np.asarray(V, dtype=np.int64)
    if operator in ("fwd_l1", "fwd_l2"):
        dx = np.zeros_like(V)
        dy = np.zeros_like(V)
        dx[:, :-1] = V[:, 1:] - V[:, :-1]
        dy[:-1, :] = V[1:, :] - V[:-1, :]
        if operator == "fwd_l1":
            return np.abs(dx) + np.abs(dy)
        return _round_sqrt(dx * dx + dy * dy)
    if operator == "sobel_l1":
        P = np.pad(V, 1, mode="edge")
        H, W = V.shape
        n = lambda dy, dx: P[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]  # noqa: E731
        gx = (n(-1, 1) + 2 * n(0, 1) + n(1, 1)) - (n(-1, -1) + 2 * n(0, -1) + n(1, -1))
        gy = (n(1, -1) + 2 * n(1, 0) + n(1, 1)) - (n(-1, -1) + 2 * n(-1, 0) + n(-1, 1))
        return (np.abs(gx) + np.abs(gy) + 2) // 4
    raise ValueError(f"unknown gradient operator {operator!r}")


def gradient_histogram(V: np.ndarray, levels: int, operator: str = "fwd_l1", rescale: str = "max"):
    """H_C(grad S) on the l image levels (Alg. 1 initialisation).

    Returns (raw, gmax, hist): raw is the 2l-1 level histogram of the gradient
    image, gmax its largest occupied level, and hist the l-level histogram.
    With rescale "max" (the default) raw level j goes to
    round-half-up(j * (l-1) / gmax) (everything to level 0 when gmax = 0);
    with "clip" it goes to min(j, l-1).  The total count stays N.
    """
    g = gradient_magnitude(V, operator)
    raw = count_histogram(g, 2 * levels - 1)
    occupied = np.nonzero(raw)[0]
    gmax = int(occupied.max()) if occupied.size else 0
    hist = np.zeros(levels, dtype=np.int64)
    if rescale == "clip":
        for j in range(2 * levels - 1):
            hist[min(j, levels - 1)] += raw[j]
        return raw, gmax, hist
    if rescale != "max":
        raise ValueError(f"unknown rescale {rescale!r}")
    if gmax == 0:
        hist[0] = raw.sum()
        return raw, gmax, hist
    for j in range(gmax + 1):
        q = (2 * (levels - 1) * j + gmax) // (2 * gmax)
        hist[q] += raw[j]
    return raw, gmax, hist


# --------------------------------------------------------------------------
# Location matrices and classification (Eqs. 7, 8, 10, 17-19)
# --------------------------------------------------------------------------

def location_vector(levels: int) -> np.ndarray:
    """Location histogram H_B: the position k/(l-1) of every level k."""
    return np.arange(levels, dtype=np.float64) / (levels - 1)


def _nearest_level(loc: np.ndarray, levels: int) -> np.ndarray:
    """argmin_k |loc - H_B(S)_k| for every entry of ``loc`` (ties: smallest k),
    evaluated literally against all l candidate levels."""
    grid = location_vector(levels)
    out = np.empty(loc.shape, dtype=np.int64)
    flat_in = loc.reshape(-1)
    flat_out = out.reshape(-1)
    step = max(1, (1 << 23) // levels)
    for s in range(0, flat_in.size, step):
        chunk = flat_in[s:s + step]
        flat_out[s:s + step] = np.argmin(np.abs(chunk[:, None] - grid[None, :]), axis=1)
    return out


@functools.lru_cache(maxsize=8)
def _classify_cached(levels: int) -> np.ndarray:
    hb = location_vector(levels)
    loc = np.outer(hb, hb)  # Eq. (7): H_B(L) x H_B(R)^T
    idx = _nearest_level(loc, levels)
    idx.setflags(write=False)
    return idx


def classify(levels: int) -> np.ndarray:
    """index(a, b) of Eq. (10): the level of S nearest to the location-matrix
    entry H_B(L)_a * H_B(R)_b (Eq. 7).  Returns an l x l int64 matrix."""
    if levels < 2:
        raise ValueError("need at least 2 levels")
    return _classify_cached(levels)


@functools.lru_cache(maxsize=8)
def _classify_enhanced_cached(levels: int, gamma: float) -> np.ndarray:
    hb = location_vector(levels)
    theta = hb ** (1.0 / gamma)  # Eq. (17)
    loc1 = np.outer(theta, hb)  # Eq. (18)
    idx1 = _nearest_level(loc1, levels)  # Eq. (19)
    idx1.setflags(write=False)
    return idx1


def classify_enhanced(levels: int, gamma: float) -> np.ndarray:
    """index_1(a, b) of Eq. (19) on the gamma-brightened location matrix of
    Eqs. (17)-(18)."""
    if not (gamma > 0 and np.isfinite(gamma)):
        raise ValueError("gamma must be positive")
    return _classify_enhanced_cached(levels, float(gamma))


# --------------------------------------------------------------------------
# Histogram-domain Retinex optimisation (Eqs. 6, 8, 10-15; Alg. 1)
# --------------------------------------------------------------------------

def init_state(hS: np.ndarray, hG: np.ndarray, init_l: str = "image"):
    """Alg. 1 initialisation in probability units: s = H_C(S)/N,
    g = H_C(grad S)/N, R^(0) = g and (our reading) L^(0) = s, or with
    init_l "uniform" L^(0) = 1/l on every level."""
    hS = np.asarray(hS, dtype=np.float64)
    hG = np.asarray(hG, dtype=np.float64)
    N = hS.sum()
    if N <= 0 or hG.sum() != N:
        raise ValueError("histograms must be non-empty and of equal mass")
    s = hS / N
    g = hG / N
    if init_l == "uniform":
        return s, g, np.full(s.size, 1.0 / s.size), g.copy()
    if init_l != "image":
        raise ValueError(f"unknown init_l {init_l!r}")
    return s, g, s.copy(), g.copy()


def weights(lv: np.ndarray, rv: np.ndarray, idx: np.ndarray):
    """Count matrix C = L R^T (Eq. 6, probability units), class totals
    d_m = sum of C over cells with index m (Eq. 8), and the weights
    K = C / d_index (Eq. 11), 0 where the class total is 0."""
    levels = lv.size
    C = np.outer(lv, rv)
    d = np.bincount(idx.ravel(), weights=C.ravel(), minlength=levels)
    dcell = d[idx]
    K = np.zeros_like(C)
    pos = dcell > 0
    K[pos] = C[pos] / dcell[pos]
    return C, d, K


def objective(lv, rv, K, s, g, idx, alpha, beta) -> float:
    """J of Eq. (10) with the weights K held fixed, in probability units
    (the paper's J in counts is N^2 times this).  Sums run over all levels."""
    S_idx = s[idx]
    fit = np.outer(lv, rv) - K * S_idx
    return float((fit ** 2).sum() + alpha * ((lv - s) ** 2).sum()
                 + beta * ((rv - g) ** 2).sum())


def update_step(lv, rv, s, g, idx, alpha, beta, K=None, update: str = "mul"):
    """One pass of the Alg. 1 loop.

    R is updated by Eq. (13) with the current L and K, L by Eq. (12) with the
    new (unnormalised) R and the same K, then both are rescaled to unit mass
    (Eqs. 15, 14).  With update "mul" (our reading) the sums weight S_index by
    K; with "div" they divide by K as printed, cells with K = 0 (an empty
    level of L or R, or an empty class) contributing nothing.  Returns a dict
    with the unnormalised and normalised iterates and the K that was used.
    """
    if K is None:
        _, _, K = weights(lv, rv, idx)
    S_idx = s[idx]
    if update == "mul":
        W = K
    elif update == "div":
        W = np.zeros_like(K)
        pos = K > 0
        W[pos] = 1.0 / K[pos]
    else:
        raise ValueError(f"unknown update {update!r}")
    # Eq. (13): R_b = (sum_a L_a K_ab S_index(a,b) + beta G_b) / (sum_a L_a^2 + beta)
    r_new = ((lv[:, None] * W * S_idx).sum(axis=0) + beta * g) / ((lv ** 2).sum() + beta)
    # Eq. (12): L_a = (sum_b R_b K_ab S_index(a,b) + alpha S_a) / (sum_b R_b^2 + alpha)
    l_new = ((r_new[None, :] * W * S_idx).sum(axis=1) + alpha * s) / ((r_new ** 2).sum() + alpha)
    return {
        "K": K,
        "r_unnorm": r_new,
        "l_unnorm": l_new,
        "r": r_new / r_new.sum(),  # Eq. (15)
        "l": l_new / l_new.sum(),  # Eq. (14)
    }


def solve(hS, hG, params: Params, record: bool = False):
    """Alg. 1: at most ``params.iters`` passes, fewer when the stopping rule
    fires (``params.eps`` > 0).

    Returns (l, r, info): the normalised illumination and reflectance
    histograms in probability units and a dict of diagnostics: "passes" (the
    passes run), "change_l" / "change_r" (per pass, the squared norm of the
    change of the normalised L / R), "stop_margin" (the smallest relative
    distance |max(change_l, change_r) - eps| / eps over the passes whose
    stopping decision was taken: how far every decision was from flipping;
    inf when eps <= 0), and with ``record`` the per-step objective values.
    """
    levels = int(params.bins)
    idx = classify(levels)
    s, g, lv, rv = init_state(hS, hG, params.init_l)
    eps = float(params.eps)
    info = {"J_before": [], "J_after_r": [], "J_after_l": [], "residual": [], "change_l": [], "change_r": []}
    margin = np.inf
    passes = 0
    _, _, K = weights(lv, rv, idx)
    for _ in range(int(params.iters)):
        step = update_step(lv, rv, s, g, idx, params.alpha, params.beta, K=K, update=params.update)
        if record:
            info["J_before"].append(objective(lv, rv, K, s, g, idx, params.alpha, params.beta))
            info["J_after_r"].append(objective(lv, step["r_unnorm"], K, s, g, idx,
                                               params.alpha, params.beta))
            info["J_after_l"].append(objective(step["l_unnorm"], step["r_unnorm"], K, s, g,
                                               idx, params.alpha, params.beta))
            info["residual"].append(max(np.abs(step["l"] - lv).max(),
                                        np.abs(step["r"] - rv).max()))
        change_l = float(((step["l"] - lv) ** 2).sum())
        change_r = float(((step["r"] - rv) ** 2).sum())
        info["change_l"].append(change_l)
        info["change_r"].append(change_r)
        lv, rv = step["l"], step["r"]
        passes += 1
        _, d, K = weights(lv, rv, idx)  # Eq. (11) for the next pass
        if record:
            tiny = d[(d > 0) & (d < 1e-30)]
            if tiny.size:
                info.setdefault("tiny_class_totals", []).append(tiny.min())
        if eps > 0 and passes < int(params.iters):
            worst = max(change_l, change_r)
            margin = min(margin, abs(worst - eps) / eps)
            if worst <= eps:  # both changes at most eps
                break
    info["passes"] = passes
    info["stop_margin"] = margin
    info["d"] = weights(lv, rv, idx)[1]
    return lv, rv, info


# --------------------------------------------------------------------------
# Histogram reprocessing (Eqs. 17-20)
# --------------------------------------------------------------------------

def target_histogram(lv, rv, npix: int, gamma: float) -> np.ndarray:
    """H_C(S~) of Eq. (20): the final count matrix N L R^T summed over the
    cells of each class of the gamma-brightened location matrix (Eq. 19)."""
    levels = lv.size
    idx1 = classify_enhanced(levels, gamma)
    C = npix * np.outer(lv, rv)
    return np.bincount(idx1.ravel(), weights=C.ravel(), minlength=levels)


# --------------------------------------------------------------------------
# Histogram matching back to pixels (end of Sec. III-C)
# --------------------------------------------------------------------------

def matching_lut(hS, target):
    """Histogram-matching map from image levels to target levels.

    The image CDF is taken at the middle of each level's pixel run,
    u(v) = (F_S(v-1) + F_S(v)) / 2, the target CDF is F~(k) = C(k) / C(l-1)
    with C the running sum of the target histogram, and
    LUT[v] = min{k : F~(k) >= u(v)}.  Taking the mid-rank keeps u strictly
    inside (0, 1) at every occupied level, so the brightest and darkest levels
    are placed by the bulk of the target mass and not by its vanishing tails.
    Also returns the distance of each decision from a flip,
    margin[v] = min(F~(LUT[v]) - u(v), u(v) - F~(LUT[v]-1)).
    """
    hS = np.asarray(hS, dtype=np.int64)
    target = np.asarray(target, dtype=np.float64)
    levels = hS.size
    N = int(hS.sum())
    cS = np.cumsum(hS)
    cS_prev = cS - hS
    u = (cS_prev + cS).astype(np.float64) / (2.0 * N)
    C = np.cumsum(target)
    Ft = C / C[-1]
    lut = np.empty(levels, dtype=np.int64)
    margin = np.empty(levels, dtype=np.float64)
    for v in range(levels):
        k = int(np.argmax(Ft >= u[v]))  # first level whose CDF reaches u[v]
        lut[v] = k
        upper = Ft[k] - u[v]
        lower = u[v] - Ft[k - 1] if k > 0 else np.inf
        margin[v] = min(upper, lower)
    return lut, margin


def equalization_lut(hS):
    """Classical histogram equalisation (Eq. 5), the comparator of the
    histogram-domain methods: level i goes to t_i = (l-1) sum_{j<=i} P_C(S)_j
    with P_C of Eq. (4), rounded to the nearest level (ties upwards).  In
    integers: t_i = floor((2 (l-1) c_i + N) / (2N)), c_i the running count."""
    hS = np.asarray(hS, dtype=np.int64)
    levels = hS.size
    N = int(hS.sum())
    if N <= 0:
        raise ValueError("empty histogram")
    c = np.cumsum(hS)
    return (2 * (levels - 1) * c + N) // (2 * N)


def remap(img: np.ndarray, lut: np.ndarray) -> np.ndarray:
    """Replace the value channel by LUT[V] keeping hue and saturation:
    out_c = round-half-up(c * LUT[V] / V); black pixels (V = 0) become grey
    LUT[0]."""
    X = img.astype(np.int64)
    V = X.max(axis=2)
    Lv = np.asarray(lut, dtype=np.int64)[V]
    out = np.empty_like(X)
    pos = V > 0
    Vp = V[pos][:, None]
    out[pos] = (2 * X[pos] * Lv[pos][:, None] + Vp) // (2 * Vp)
    out[~pos] = Lv[~pos][:, None]
    return out.astype(img.dtype)


# --------------------------------------------------------------------------
# Whole pipeline
# --------------------------------------------------------------------------

def enhance(img: np.ndarray, params: Params = Params(), record: bool = False):
    """Image -> enhanced image with every intermediate (dict)."""
    levels = int(params.bins)
    if levels not in (256, 1024) and levels & (levels - 1):
        raise ValueError("bins must be a power of two")
    V = value_channel(img)
    if V.max(initial=0) >= levels:
        raise ValueError("pixel value exceeds the level range")
    npix = V.size
    hS = count_histogram(V, levels)
    graw, gmax, hG = gradient_histogram(V, levels, params.grad_op, params.grad_rescale)
    lv, rv, info = solve(hS, hG, params, record=record)
    target = target_histogram(lv, rv, npix, params.gamma)
    lut, margin = matching_lut(hS, target)
    out = remap(img, lut)
    return {
        "V": V, "hS": hS, "graw": graw, "gmax": gmax, "hG": hG, "passes": info["passes"],
        "l": lv, "r": rv, "illum": npix * lv, "refl": npix * rv,
        "target": target, "lut": lut, "margin": margin, "out": out,
        "npix": npix, "info": info,
    }
