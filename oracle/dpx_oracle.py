"""FP64 CPU oracle for multi-wavelength diffractive propagation and its gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run this module.  The product path
(the HIP library and its Python binding) never calls it, and this module
imports nothing from the product package.

What it computes (paper, Section 4 "Optical forward model of
wavelength-multiplexed diffractive systems", Eq. 1, 2, 4, 5; problem
statement in Section 2 and the Fig. 1 caption):

* every wavelength lambda_w starts from the input field u_in (unit plane wave
  by default: the paper's "uniform input fields"),
* each of the K layers multiplies the field by the transmission of Eq. 1,
  t = exp(-2 pi kappa h / lambda) * exp(+j 2 pi (n - n_m) h / lambda),
  h being the total thickness of Eq. 2 (the sign reading is explained below),
* the field then travels the gap z_l by the Rayleigh-Sommerfeld convolution of
  Eq. 4/5, evaluated here by the angular spectrum: zero-pad N -> M = pad*N
  (centred), 2-D DFT, multiply by H = exp(+j 2 pi z sqrt(q)) with
  q = (n_m/lambda)^2 - fx^2 - fy^2 where q > 0 and H = 0 elsewhere (the
  evanescent part is cut), inverse DFT (1/M^2), crop back to N x N,
* the output intensity O_w = |o_w|^2 is cropped to the central F x F
  field of view and summed over bin x bin blocks into a T x T image,
* loss: per wavelength the intensity and the target are each normalised to
  unit sum, the mean squared difference over the T^2 pixels is taken, and the
  mean over wavelengths is the loss (the paper's MSE-based loss; its exact
  form lives in a supplement that is not available),
* gradient: reverse-mode (adjoint) pass written by hand in FP64.

Readings of the paper used here (each also listed with the design notes):

* Eq. 1 prints exp(-j 2 pi (n - n_air) h / lambda) next to the absorption
  factor exp(-2 pi kappa h / lambda); that absorption sign is only consistent
  with the exp(+j k r) outgoing-wave convention of Eq. 4, under which optical
  path adds phase exp(+j 2 pi (n - n_air) h / lambda).  We use +j.  The
  printed sign equals ours with h -> -h (kappa = 0).
* "n" in Eq. 4 is the index of the gap medium n_m (air, n_m = 1); n_air in
  Eq. 1 is the same n_m.
* Eq. 5 has no area element; the direct Rayleigh-Sommerfeld sum below
  multiplies by dx^2 so that it approximates the continuous integral.  The
  angular spectrum needs none (unitary DFT pair).
* The field outside the N x N layer aperture is dropped after every gap.
* Input plane: the uniform illumination passes the input aperture (u_in) and
  reaches layer 1 after the optional gap z_in (the Fig. 1 schematic, the
  input plane being one of the planes connected by diffraction); z_in = 0
  means u_in is the field at layer 1.
* Band-limited angular spectrum (an alternative transfer function, off
  unless a design sets band_limited): H is set to zero where the sampled
  phase would alias (band_limit below).
* Phase-only layers (Eq. 3) are the thickness model with a unit index
  contrast and no dispersion; phase_only_transmission states them directly.
* Misalignment (Section 2, the "vaccination" against lateral and axial
  displacements): gap l may be lengthened by dz_l and may translate the field
  it delivers by (sx_l, sy_l), a factor exp(-j 2 pi (fx sx + fy sy)) on H.
  Layer offsets D_l map to gap translations D_l - D_(l+1) with the output
  plane fixed; the input field moves with the first layer.

DFT conventions: forward kernel exp(-2 pi j k n / M) with exact integer
reduction (k n mod M) before the angle is formed, unnormalised; the inverse
carries 1/M^2.  Frequencies are fx = k'/(M dx) with k' the signed index in
[-M/2, M/2).

Two evaluation modes for the 2-D DFT: ``"naive"`` forms the DFT matrix from
its definition and applies it with matrix products; ``"fft"`` calls
``numpy.fft`` (pocketfft, FP64).  Both are pinned against each other and
against closed forms by the oracle tests.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


# ------------------------------------------------------------------------------------------
# Discrete Fourier transform (Section 4: the gap propagation is a linear shift-invariant
# convolution, Eq. 5; here evaluated through the DFT).
# ------------------------------------------------------------------------------------------

def signed_index(M: int) -> np.ndarray:
    """k' = k for k < M/2, k - M otherwise (the order numpy.fft.fftfreq uses)."""
    k = np.arange(M, dtype=np.int64)
    return np.where(k < (M + 1) // 2, k, k - M)


def dft_matrix(M: int) -> np.ndarray:
    """F[k, n] = exp(-2 pi j ((k n) mod M) / M)."""
    n = np.arange(M, dtype=np.int64)
    idx = np.outer(n, n) % M
    return np.exp(-1j * TWO_PI * idx.astype(np.float64) / M)


_DFT_CACHE: dict[int, np.ndarray] = {}


def _dft(M):
    F = _DFT_CACHE.get(M)
    if F is None:
        F = dft_matrix(M)
        _DFT_CACHE[M] = F
    return F


def dft2(U: np.ndarray, mode: str = "naive") -> np.ndarray:
    """Unnormalised 2-D DFT over the last two axes (square)."""
    if mode == "fft":
        return np.fft.fft2(U, axes=(-2, -1))
    F = _dft(U.shape[-1])
    return F @ U @ F.T


def idft2(V: np.ndarray, mode: str = "naive") -> np.ndarray:
    """Inverse 2-D DFT with the 1/M^2 factor."""
    if mode == "fft":
        return np.fft.ifft2(V, axes=(-2, -1))
    M = V.shape[-1]
    G = np.conj(_dft(M))
    return (G @ V @ G.T) / float(M * M)


# ------------------------------------------------------------------------------------------
# Transfer function of the gap (Eq. 4 in the spectral domain).
# ------------------------------------------------------------------------------------------

def spatial_frequencies(M: int, dx: float) -> np.ndarray:
    return signed_index(M).astype(np.float64) / (M * dx)


def band_limit(M: int, dx: float, wl: float, n_medium: float, z: float) -> float:
    """Band limit of the sampled transfer function (Matsushima and Shimobaba's band-limited
    angular spectrum): the phase 2 pi z sqrt(k^2 - f^2), k = n_m / lambda, sampled every
    1 / (M dx) in f, changes by at most pi between samples while its local frequency
    z |f| / sqrt(k^2 - f^2) stays within M dx / 2, i.e. for |f| <= k / sqrt((2 z / (M dx))^2 + 1)."""
    return (n_medium / wl) / np.sqrt((2.0 * z / (M * dx)) ** 2 + 1.0)


def transfer_function(M: int, dx: float, wl: float, n_medium: float, z: float,
                      shift=(0.0, 0.0), band_limited: bool = False) -> np.ndarray:
    """H[ky, kx] = exp(+j 2 pi z sqrt(q)) for q = (n_m/lambda)^2 - fx^2 - fy^2 > 0, else 0.

    With shift = (sx, sy) in metres H is multiplied by exp(-j 2 pi (fx sx + fy sy)): the
    propagated field is translated by (+sx, +sy) (Fourier shift theorem), which is how a
    lateral misalignment of the following element enters (Section 2, misalignment)."""
    f = spatial_frequencies(M, dx)
    q = (n_medium / wl) ** 2 - f[None, :] ** 2 - f[:, None] ** 2
    prop = q > 0.0
    root = np.sqrt(np.where(prop, q, 0.0))
    H = np.where(prop, np.exp(1j * TWO_PI * z * root), 0.0)
    if band_limited:
        lim = band_limit(M, dx, wl, n_medium, z)
        H = np.where((np.abs(f[None, :]) <= lim) & (np.abs(f[:, None]) <= lim), H, 0.0)
    sx, sy = float(shift[0]), float(shift[1])
    if sx != 0.0 or sy != 0.0:
        H = H * np.exp(-1j * TWO_PI * (f[None, :] * sx + f[:, None] * sy))
    return H


def pad_centered(u: np.ndarray, M: int) -> np.ndarray:
    N = u.shape[-1]
    o = (M - N) // 2
    U = np.zeros(u.shape[:-2] + (M, M), dtype=np.complex128)
    U[..., o:o + N, o:o + N] = u
    return U


def crop_centered(U: np.ndarray, N: int) -> np.ndarray:
    M = U.shape[-1]
    o = (M - N) // 2
    return U[..., o:o + N, o:o + N]


def propagate(u: np.ndarray, pad: int, dx: float, wl: float, n_medium: float, z: float,
              mode: str = "naive", adjoint: bool = False, shift=(0.0, 0.0),
              band_limited: bool = False) -> np.ndarray:
    """One gap: pad -> DFT2 -> x H -> IDFT2 -> crop.  ``adjoint`` applies the Hermitian
    adjoint of that linear map, which is the same chain with conj(H)."""
    N = u.shape[-1]
    M = pad * N
    H = transfer_function(M, dx, wl, n_medium, z, shift, band_limited)
    if adjoint:
        H = np.conj(H)
    V = idft2(H * dft2(pad_centered(u, M), mode), mode)
    return crop_centered(V, N)


# ------------------------------------------------------------------------------------------
# Layer transmission (Eq. 1, 2).
# ------------------------------------------------------------------------------------------

def layer_constants(wl: float, n_mat: float, kappa: float, n_medium: float):
    """(c_t, c_a): phase and absorption per metre of thickness, Eq. 1."""
    c_t = TWO_PI * (n_mat - n_medium) / wl
    c_a = TWO_PI * kappa / wl
    return c_t, c_a


def transmission(h: np.ndarray, wl: float, n_mat: float, kappa: float, n_medium: float):
    c_t, c_a = layer_constants(wl, n_mat, kappa, n_medium)
    h = np.asarray(h, dtype=np.float64)
    return np.exp(-c_a * h) * np.exp(1j * c_t * h)


# ------------------------------------------------------------------------------------------
# Cascade, intensity, loss, gradient.
# ------------------------------------------------------------------------------------------

def gap(design: dict, l: int):
    """Gap l (after layer l; the last one ends at the output plane) as (length, (sx, sy)):
    z_l plus the axial jitter dz_l, and the lateral translation of the field it delivers.
    The optional design keys dz, shift_x, shift_y hold one value per gap in metres."""
    def at(key):
        v = design.get(key)
        return 0.0 if v is None else float(v[l])
    return float(design["z"][l]) + at("dz"), (at("shift_x"), at("shift_y"))


def gap_shifts_from_layer_offsets(D: np.ndarray) -> np.ndarray:
    """Lateral offsets D[l] = (Dx, Dy) of layers 0..K-1 (output plane fixed) -> the field
    translation of every gap.  In the frame of a displaced element its transmission is the
    undisplaced one and the incoming field appears translated by -D; propagation commutes with
    translations, so gap l translates by D[l] - D[l+1], with D[K] = 0.  The input field is
    taken in the frame of layer 0 (the aperture moves with the first layer)."""
    D = np.asarray(D, np.float64)
    nxt = np.vstack([D[1:], np.zeros((1, 2))])
    return D - nxt


def gap_jitter_from_layer_offsets(Dz: np.ndarray) -> np.ndarray:
    """Axial offsets Dz[l] of layers 0..K-1 (output plane fixed) -> the change of every gap
    length: gap l runs from layer l to layer l+1 (or the output plane), so it changes by
    Dz[l+1] - Dz[l], with Dz[K] = 0."""
    Dz = np.asarray(Dz, np.float64)
    return np.append(Dz[1:], 0.0) - Dz


def quantize_heights(h: np.ndarray, h_max: float, bits: int) -> np.ndarray:
    """Phase bit depth B (Section 2, fabrication limits): 2^B thickness levels k h_max / (2^B - 1),
    k = 0 .. 2^B - 1, each height taken to the nearest level (ties to even), heights outside
    [0, h_max] to the end levels.  The level index is an integer decided by floating point, so it
    is decided in single precision: k = rint(h * s) with s = fl32((2^B - 1) / h_max), the level
    value fl32(k) * fl32(h_max / (2^B - 1))."""
    levels = (1 << bits) - 1
    s = np.float32(levels / h_max)
    step = np.float32(h_max / levels)
    k = np.rint(np.asarray(h, np.float32) * s)
    k = np.clip(k, np.float32(0), np.float32(levels))
    return (k * step).astype(np.float32)


def phase_only_transmission(phi: np.ndarray, wl: float, lam_ref: float) -> np.ndarray:
    """Eq. 3, a phase-only pixel (the spatial light modulator of the experiment), with the sign
    reading of Eq. 1 (+j): exp(+j phi lambda_ref / lambda), phi being the phase at lambda_ref of a
    fixed optical path."""
    return np.exp(1j * np.asarray(phi, np.float64) * (lam_ref / wl))


def _kappa(design, w):
    k = design.get("kappa")
    return 0.0 if k is None else float(k[w])


def fov_slice(design):
    N, F = design["n"], design["fov"]
    a = (N - F) // 2
    return slice(a, a + F)


def bin_sum(x: np.ndarray, b: int) -> np.ndarray:
    F = x.shape[-1]
    T = F // b
    return x.reshape(x.shape[:-2] + (T, b, T, b)).sum(axis=(-3, -1))


def forward(design: dict, h: np.ndarray, u_in=None, mode: str = "naive", keep: bool = False,
            wavelengths=None):
    """Intensity images I[w, T, T] for every wavelength (Eq. 5 recursion, then |o|^2 on the
    field of view).  With ``keep`` also return the per-layer fields after the transmission
    multiply (v[w, l]) and the output field on the field of view (o[w])."""
    N, K = design["n"], design["layers"]
    ws = range(design["n_wl"]) if wavelengths is None else list(wavelengths)
    fs = fov_slice(design)
    b = design["bin"]
    T = design["fov"] // b
    h64 = np.asarray(h, dtype=np.float64)
    u0 = np.ones((N, N), np.complex128) if u_in is None else np.asarray(u_in, np.complex128)
    out = np.zeros((len(ws), T, T), dtype=np.float64)
    vs = np.zeros((len(ws), K, N, N), np.complex128) if keep else None
    os_ = np.zeros((len(ws), design["fov"], design["fov"]), np.complex128) if keep else None
    z_in = float(design.get("z_in") or 0.0)
    bl = bool(design.get("band_limited"))
    for i, w in enumerate(ws):
        wl, nm = float(design["wl"][w]), float(design["n_mat"][w])
        u = u0
        if z_in > 0.0:
            # the input plane (u_in, e.g. the illumination aperture) lies z_in before layer 1
            u = propagate(u0, design["pad"], design["dx"], wl, design["n_medium"], z_in, mode,
                          band_limited=bl)
        for l in range(K):
            v = transmission(h64[l], wl, nm, _kappa(design, w), design["n_medium"]) * u
            if keep:
                vs[i, l] = v
            z, sh = gap(design, l)
            u = propagate(v, design["pad"], design["dx"], wl, design["n_medium"], z, mode, shift=sh,
                          band_limited=bl)
        o = u[fs, fs]
        if keep:
            os_[i] = o
        out[i] = bin_sum(np.abs(o) ** 2, b)
    if keep:
        return out, vs, os_
    return out


def forward_phase_only(design: dict, phi: np.ndarray, lam_ref: float, u_in=None, mode: str = "naive",
                       wavelengths=None):
    """Intensity images of a cascade of phase-only layers (Eq. 3, the spatial light modulators of
    the experiment): layer l multiplies the field by phase_only_transmission(phi[l]) at each
    wavelength, then the gap of Eq. 4/5 follows exactly as in ``forward`` (same padding, cut,
    crop and field of view).  phi [K, N, N] radians at lam_ref.  No input gap, no misalignment."""
    N, K = design["n"], design["layers"]
    ws = range(design["n_wl"]) if wavelengths is None else list(wavelengths)
    fs = fov_slice(design)
    b = design["bin"]
    T = design["fov"] // b
    u0 = np.ones((N, N), np.complex128) if u_in is None else np.asarray(u_in, np.complex128)
    out = np.zeros((len(ws), T, T), dtype=np.float64)
    for i, w in enumerate(ws):
        wl = float(design["wl"][w])
        u = u0
        for l in range(K):
            v = phase_only_transmission(phi[l], wl, lam_ref) * u
            z, sh = gap(design, l)
            u = propagate(v, design["pad"], design["dx"], wl, design["n_medium"], z, mode, shift=sh)
        out[i] = bin_sum(np.abs(u[fs, fs]) ** 2, b)
    return out


def loss(I: np.ndarray, tau: np.ndarray):
    """L = (1/W) sum_w mean_p (I_w,p / S_w - tau_w,p / sum tau_w)^2 and dL/dI.

    A wavelength whose intensity (or target) sums to zero contributes a zero ratio and a
    zero gradient."""
    I = np.asarray(I, np.float64)
    tau = np.asarray(tau, np.float64)
    W = I.shape[0]
    P = I.shape[-1] * I.shape[-2]
    S = I.sum(axis=(1, 2))
    St = tau.sum(axis=(1, 2))
    Ih = np.where(S[:, None, None] > 0, I / np.where(S > 0, S, 1.0)[:, None, None], 0.0)
    th = np.where(St[:, None, None] > 0, tau / np.where(St > 0, St, 1.0)[:, None, None], 0.0)
    d = Ih - th
    per_wl = (d * d).sum(axis=(1, 2)) / P
    L = per_wl.sum() / W
    inner = (d * Ih).sum(axis=(1, 2))
    g = 2.0 / (W * P) * (d - inner[:, None, None])
    g = np.where(S[:, None, None] > 0, g / np.where(S > 0, S, 1.0)[:, None, None], 0.0)
    return float(L), g, per_wl


def grad(design: dict, h: np.ndarray, u_in, dl_di: np.ndarray, mode: str = "naive",
         wavelengths=None):
    """dL/dh[l, y, x] for the given dL/dI[w, T, T] (summed over wavelengths in index order).

    Wirtinger convention: g = dL/dRe(u) + j dL/dIm(u).  Output seed g = 2 (dL/dI) o on the
    field of view.  Back through a gap: g <- P^H g.  At layer l with v = t u:
    dL/dh += -c_t Im(conj(g) v) - c_a Re(conj(g) v), then g <- conj(t) g."""
    N, K = design["n"], design["layers"]
    ws = list(range(design["n_wl"])) if wavelengths is None else list(wavelengths)
    fs = fov_slice(design)
    b = design["bin"]
    _, vs, os_ = forward(design, h, u_in, mode, keep=True, wavelengths=ws)
    h64 = np.asarray(h, dtype=np.float64)
    dh = np.zeros((K, N, N), np.float64)
    for i, w in enumerate(ws):
        wl, nm = float(design["wl"][w]), float(design["n_mat"][w])
        c_t, c_a = layer_constants(wl, nm, _kappa(design, w), design["n_medium"])
        dI = np.repeat(np.repeat(np.asarray(dl_di[i], np.float64), b, axis=0), b, axis=1)
        g = np.zeros((N, N), np.complex128)
        g[fs, fs] = 2.0 * dI * os_[i]
        for l in range(K - 1, -1, -1):
            z, sh = gap(design, l)
            g = propagate(g, design["pad"], design["dx"], wl, design["n_medium"], z, mode,
                          adjoint=True, shift=sh, band_limited=bool(design.get("band_limited")))
            p = np.conj(g) * vs[i, l]
            dh[l] += -c_t * p.imag - c_a * p.real
            g = np.conj(transmission(h64[l], wl, nm, _kappa(design, w), design["n_medium"])) * g
    return dh


def loss_of_heights(design, h, u_in, tau, mode="naive", wavelengths=None):
    I = forward(design, h, u_in, mode, wavelengths=wavelengths)
    t = tau if wavelengths is None else np.asarray(tau)[list(wavelengths)]
    return loss(I, t)[0]


def fd_pixels(design, h, u_in, tau, pixels, delta, mode="naive"):
    """Central differences of the loss w.r.t. single heights h[l, y, x] (FP64)."""
    h64 = np.asarray(h, dtype=np.float64)
    out = np.zeros(len(pixels))
    for i, (l, y, x) in enumerate(pixels):
        hp = h64.copy()
        hm = h64.copy()
        hp[l, y, x] += delta
        hm[l, y, x] -= delta
        out[i] = (loss_of_heights(design, hp, u_in, tau, mode)
                  - loss_of_heights(design, hm, u_in, tau, mode)) / (2 * delta)
    return out


def fd_direction(design, h, u_in, tau, v, delta, mode="naive"):
    """Central difference of the loss along the direction v (same shape as h)."""
    h64 = np.asarray(h, dtype=np.float64)
    lp = loss_of_heights(design, h64 + delta * v, u_in, tau, mode)
    lm = loss_of_heights(design, h64 - delta * v, u_in, tau, mode)
    return (lp - lm) / (2 * delta)


# ------------------------------------------------------------------------------------------
# Direct Rayleigh-Sommerfeld sum (Eq. 4, 5) for tiny grids.
# ------------------------------------------------------------------------------------------

def rs_kernel(dxs: np.ndarray, dys: np.ndarray, z: float, wl: float, n_medium: float):
    """w = z / r^2 (1/(2 pi r) + n / (j lambda)) exp(j 2 pi n r / lambda), Eq. 4."""
    r = np.sqrt(dxs * dxs + dys * dys + z * z)
    return z / (r * r) * (1.0 / (TWO_PI * r) + n_medium / (1j * wl)) * np.exp(
        1j * TWO_PI * n_medium * r / wl)


def rs_direct(u: np.ndarray, dx: float, wl: float, n_medium: float, z: float) -> np.ndarray:
    """u_out(p) = sum_s u(s) w(p - s) dx^2 on the same N x N lateral grid, O(N^4)."""
    N = u.shape[-1]
    d = (np.arange(2 * N - 1) - (N - 1)).astype(np.float64) * dx
    Kd = rs_kernel(d[None, :], d[:, None], z, wl, n_medium) * dx * dx   # [dy, dx]
    # Toeplitz blocks T[dy][px, sx] = Kd[dy, px - sx + N - 1]
    px = np.arange(N)
    cols = px[:, None] - px[None, :] + N - 1
    T = Kd[:, cols]                                                      # [2N-1, N, N]
    out = np.zeros((N, N), np.complex128)
    sy = np.arange(N)
    for py in range(N):
        blocks = T[py - sy + N - 1]                                      # [N(sy), N(px), N(sx)]
        out[py] = np.einsum("spk,sk->p", blocks, u)
    return out


# ------------------------------------------------------------------------------------------
# Training support (Section 4, "Data preparation and other implementation details": Adam with
# the optimizer library's default parameters, learning rate 0.001; Section 2: output PSNR per
# image-wavelength pair).  Readings: the heights are kept in [0, h_max] through an
# unconstrained variable, h = h_max * sigmoid(theta) (the paper does not say how its bound is
# enforced), and PSNR is the textbook one on the unit-sum normalised images with the target's
# peak (the paper's convention is in its missing supplement).
# ------------------------------------------------------------------------------------------
ADAM_DEFAULTS = dict(lr=1e-3, b1=0.9, b2=0.999, eps=1e-8)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def adam_update(g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma and Ba): moment estimates, bias correction by 1 - b^step, and the step
    -lr * m_hat / (sqrt(v_hat) + eps).  Returns (delta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    return -lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adam_sigmoid_step(theta, dl_dh, m, v, step, h_max, **adam):
    """One step on theta given dL/dh for h = h_max sigmoid(theta): chain rule
    dL/dtheta = dL/dh * h_max s (1 - s), Adam on theta.  Returns (theta, h, m, v)."""
    s = sigmoid(theta)
    g = dl_dh * h_max * s * (1.0 - s)
    delta, m, v = adam_update(g, m, v, step, **{**ADAM_DEFAULTS, **adam})
    theta = theta + delta
    return theta, h_max * sigmoid(theta), m, v


def psnr(I: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Per wavelength: 10 log10(max tau_hat^2 / mean (I_hat - tau_hat)^2), both images
    normalised to unit sum (a zero sum normalises to zero, as in the loss)."""
    I = np.asarray(I, np.float64)
    tau = np.asarray(tau, np.float64)
    W = I.shape[0]
    out = np.empty(W)
    for w in range(W):
        S, St = I[w].sum(), tau[w].sum()
        a = I[w] / S if S > 0 else np.zeros_like(I[w])
        b = tau[w] / St if St > 0 else np.zeros_like(tau[w])
        mse = np.mean((a - b) ** 2)
        out[w] = np.inf if mse == 0 else 10.0 * np.log10(b.max() ** 2 / mse)
    return out


def channel_swap(psnr_per_wl: np.ndarray, wl: np.ndarray) -> np.ndarray:
    """Dynamic channel swapping (Section 2): images sorted by PSNR, highest first, are
    reassigned to the wavelengths taken from the longest down.  Returns src such that the new
    target of wavelength w is the old target of wavelength src[w]."""
    by_psnr = np.argsort(-np.asarray(psnr_per_wl), kind="stable")
    by_length = np.argsort(-np.asarray(wl), kind="stable")
    src = np.empty(len(wl), dtype=np.int64)
    src[by_length] = by_psnr
    return src
