"""Seeded synthetic inputs for the messenger Wiener filter.

This module draws the random inputs (signal alm, noise, hit maps, masks) and
builds the power spectra and cooling schedules of the synthetic workloads. It
holds none of the filter's arithmetic: callers pass in the pixel angles of
their own HEALPix geometry, and turn the drawn signal alm into a map with their
own synthesis. Both the GPU path and its CPU checker take their inputs from
here, so they see identical bytes.

The paper's data (WMAP7 V band with the extended masks, Sect. 3) are not
available; these recipes stand in for them with the same structure: a CMB-like
power spectrum, anisotropic white pixel noise, and a galactic-plane cut plus
point-source holes.

Random streams: numpy PCG64 seeded by SeedSequence([seed, stream]) with
stream 0 = signal, 1 = noise, 2 = noise model / mask (model_seed), 3 and 4 = the
unit draws of constrained realisations (SeedSequence([seed, map, 3]) per map for
the alm draws, [seed, 4] for the pixel draws).
"""
import numpy as np

MUK = 1.0          # maps are in micro-kelvin
NEP_GAL_L_DEG = 96.38    # north ecliptic pole in galactic coordinates
NEP_GAL_B_DEG = 29.81


def rng(seed, stream):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


# ------------------------------------------------------------------ spectra
def cl_power_law(lmax, amp=1e3):
    """C_l = amp / (l (l+1)) for l >= 2, C_0 = C_1 = 0 (micro-K^2)."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    cl[2:] = amp / (l[2:] * (l[2:] + 1.0))
    return cl


def cl_satellite(lmax, amp=1e3, fwhm_arcmin=13.0, peaks=(220.0, 540.0, 800.0),
                 peak_amp=0.6, peak_width=60.0):
    """Power law with three Gaussian bumps, times a Gaussian beam b_l^2."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    bump = np.ones(lmax + 1)
    for lk in peaks:
        bump += peak_amp * np.exp(-(l - lk) ** 2 / (2.0 * peak_width ** 2))
    sigma_b = np.radians(fwhm_arcmin / 60.0) / np.sqrt(8.0 * np.log(2.0))
    beam2 = np.exp(-l * (l + 1.0) * sigma_b ** 2)
    cl[2:] = amp / (l[2:] * (l[2:] + 1.0)) * bump[2:] * beam2[2:]
    return cl


# ------------------------------------------------------------------ draws
def random_alm(cl, lmax, seed):
    """Gaussian alm of a real field with spectrum cl, packed m-major
    (index m*(2*lmax+1-m)/2 + l): a_l0 = sqrt(C_l) g, a_lm = sqrt(C_l/2)(g1 + i g2)."""
    g = rng(seed, 0) if np.isscalar(seed) else np.random.Generator(
        np.random.PCG64(np.random.SeedSequence([int(x) for x in seed])))
    cl = np.asarray(cl, dtype=np.float64)
    out = []
    for m in range(lmax + 1):
        sd = np.sqrt(cl[m:lmax + 1])
        if m == 0:
            out.append(sd * g.standard_normal(lmax + 1) + 0j)
        else:
            re = g.standard_normal(lmax + 1 - m)
            im = g.standard_normal(lmax + 1 - m)
            out.append(sd * np.sqrt(0.5) * (re + 1j * im))
    return np.concatenate(out)


def noise_draw(sigma2, seed):
    """n_p = sigma_p g_p (drawn everywhere, also where the pixel is masked)."""
    return np.sqrt(sigma2) * rng(seed, 1).standard_normal(np.size(sigma2))


def fluctuation_draws(npix, lmax, seed, nmaps=1):
    """Unit draws of a constrained realisation, one set per map: xi, packed alm with
    E|xi_lm|^2 = 1 (real N(0,1) at m = 0, (g1 + i g2)/sqrt 2 above), from stream 3;
    eta, N(0,1) per pixel, from stream 4. Shapes [nmaps, N_lm] and [nmaps, npix]."""
    ones = np.ones(lmax + 1)
    xi = np.stack([random_alm(ones, lmax, (seed, i, 3)) for i in range(nmaps)])
    g = rng(seed, 4)
    eta = g.standard_normal((nmaps, npix))
    return xi, eta


def unit_vectors(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def ecliptic_cos_colatitude(theta, phi):
    """cos of the ecliptic colatitude of galactic (theta, phi) directions."""
    lp = np.radians(NEP_GAL_L_DEG)
    bp = np.radians(NEP_GAL_B_DEG)
    nep = np.array([np.cos(bp) * np.cos(lp), np.cos(bp) * np.sin(lp), np.sin(bp)])
    return unit_vectors(theta, phi) @ nep


def galactic_cut(theta, bcut_deg):
    """True where |galactic latitude| < bcut (masked)."""
    return np.abs(0.5 * np.pi - theta) < np.radians(bcut_deg)


def disc_holes(theta, phi, ndisc, radius_deg, model_seed):
    """True inside any of `ndisc` discs with centres uniform on the sphere."""
    g = rng(model_seed, 2)
    cz = g.uniform(-1.0, 1.0, ndisc)
    cphi = g.uniform(0.0, 2.0 * np.pi, ndisc)
    centres = unit_vectors(np.arccos(cz), cphi)
    v = unit_vectors(theta, phi)
    r = np.radians(radius_deg)
    cosr = np.cos(r)
    hole = np.zeros(theta.size, dtype=bool)
    if np.all(np.diff(theta) >= 0):
        # RING order sorts pixels by colatitude: only the band |theta - theta_c| <= r
        # (plus a margin far above rounding) can lie inside a disc
        ctheta = np.arccos(cz)
        lo = np.searchsorted(theta, ctheta - r - 1e-6, side="left")
        hi = np.searchsorted(theta, ctheta + r + 1e-6, side="right")
        for c, a, b in zip(centres, lo, hi):
            hole[a:b] |= (v[a:b] @ c) > cosr
    else:
        for c in centres:
            hole |= (v @ c) > cosr
    return hole


# ------------------------------------------------------------------ workloads
def geometric_schedule(lam0, n_cool, n_final):
    """lambda_k = lam0**(1 - k/n_cool) for k < n_cool, then n_final sweeps at 1."""
    k = np.arange(n_cool)
    return np.concatenate([lam0 ** (1.0 - k / n_cool), np.ones(n_final)])


def small_band_case(theta, lmax, seed=0, model_seed=0):
    """Nside-16-style case: C_l = 1e3/(l(l+1)); sigma_p^2 = (30 muK)^2 / h_p with
    h_p = exp(0.5 g_p); equatorial band |theta - pi/2| < 0.35 rad masked;
    schedule 40 geometric steps 1e4 -> 1 then 100 sweeps at 1."""
    lmax = int(lmax)
    cl = cl_power_law(lmax)
    h = np.exp(0.5 * rng(model_seed, 2).standard_normal(theta.size))
    sigma2 = (30.0 * MUK) ** 2 / h
    mask = np.abs(theta - 0.5 * np.pi) < 0.35
    return _finish(cl, sigma2, mask, lmax, seed, geometric_schedule(1e4, 40, 100))


def satellite_model(theta, phi, lmax, model_seed=0, nobs_scale=1.0, bcut_deg=15.0, ndisc=500,
                    disc_deg=0.5, sigma0_muk=2200.0, n_cool=30, n_final=50):
    """Shared part of the satellite-style case: beam-smoothed bumpy spectrum;
    sigma_p^2 = sigma0^2 / N_obs with N_obs = 300 (1 + 2 |cos theta_ecl|^4)
    lognormal(0, 0.2) (times nobs_scale); mask |b| < bcut plus `ndisc` discs of
    radius disc_deg; schedule n_cool geometric steps 1e4 -> 1, then n_final at 1."""
    lmax = int(lmax)
    cl = cl_satellite(lmax)
    ce = ecliptic_cos_colatitude(theta, phi)
    g = rng(model_seed, 2)
    nobs = 300.0 * (1.0 + 2.0 * np.abs(ce) ** 4) * np.exp(0.2 * g.standard_normal(theta.size))
    nobs *= nobs_scale
    sigma2 = (sigma0_muk * MUK) ** 2 / nobs
    mask = galactic_cut(theta, bcut_deg)
    if ndisc:
        mask |= disc_holes(theta, phi, ndisc, disc_deg, model_seed + 1)
    return {"cl": cl, "sigma2": sigma2, "mask": mask, "ninv": np.where(mask, 0.0, 1.0 / sigma2),
            "schedule": geometric_schedule(1e4, n_cool, n_final), "lmax": lmax}


def draw(model, seed):
    """Signal alm and noise of one simulation of a shared model."""
    return {"signal_alm": random_alm(model["cl"], model["lmax"], seed),
            "noise": noise_draw(model["sigma2"], seed)}


def satellite_case(theta, phi, lmax, seed=0, model_seed=0, **kw):
    """Satellite-style case (model + one draw)."""
    c = dict(satellite_model(theta, phi, lmax, model_seed=model_seed, **kw))
    c.update(draw(c, seed))
    return c


def uniform_fullsky_case(npix, lmax, sigma_muk=30.0, seed=0, n_sweeps=3):
    """Full sky, uniform noise: every pixel observed with the same variance."""
    cl = cl_power_law(lmax)
    sigma2 = np.full(npix, (sigma_muk * MUK) ** 2)
    mask = np.zeros(npix, dtype=bool)
    return _finish(cl, sigma2, mask, lmax, seed, geometric_schedule(1e4, n_sweeps, 0)
                   if n_sweeps else np.ones(1))


def _finish(cl, sigma2, mask, lmax, seed, schedule):
    ninv = np.where(mask, 0.0, 1.0 / sigma2)
    return {
        "cl": cl,
        "ninv": ninv,
        "mask": mask,
        "sigma2": sigma2,
        "signal_alm": random_alm(cl, lmax, seed),
        "noise": noise_draw(sigma2, seed),
        "schedule": schedule,
        "lmax": lmax,
    }


# ------------------------------------------------------------------ polarisation (T, Q, U)
def cl_pol(cl_tt, e_frac=0.05, b_frac=0.01, te_corr=0.5, te_period=150.0):
    """Four spectra [TT, EE, BB, TE] from a temperature spectrum: EE = e_frac TT,
    BB = b_frac EE, TE = rho_l sqrt(TT EE) with rho_l = te_corr cos(pi l / te_period)
    (|rho| < 1 keeps every 2x2 TE block positive definite). E and B start at l = 2."""
    tt = np.asarray(cl_tt, dtype=np.float64)
    l = np.arange(tt.size, dtype=np.float64)
    ee = e_frac * tt
    bb = b_frac * ee
    te = te_corr * np.cos(np.pi * l / te_period) * np.sqrt(tt * ee)
    ee[:2] = bb[:2] = te[:2] = 0.0
    return np.stack([tt, ee, bb, te])


def random_alm_pol(cl4, lmax, seed):
    """Gaussian [T, E, B] alm with the 3x3 spectrum of cl4 (signal stream of `seed`):
    T = sqrt(TT) g1, E = TE/sqrt(TT) g1 + sqrt(EE - TE^2/TT) g2, B = sqrt(BB) g3, each g
    real at m = 0 and (g' + i g'')/sqrt 2 above, drawn m by m in packed order."""
    tt, ee, bb, te = (np.asarray(c, dtype=np.float64) for c in cl4)
    g = rng(seed, 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        c_te = np.where(tt > 0, te / np.sqrt(np.where(tt > 0, tt, 1.0)), 0.0)
        c_ee = np.sqrt(np.maximum(ee - np.where(tt > 0, te * te / np.where(tt > 0, tt, 1.0), 0.0), 0.0))
    out = [[], [], []]
    for m in range(lmax + 1):
        n = lmax + 1 - m
        if m == 0:
            g1, g2, g3 = (g.standard_normal(n) + 0j for _ in range(3))
        else:
            g1, g2, g3 = ((g.standard_normal(n) + 1j * g.standard_normal(n)) * np.sqrt(0.5) for _ in range(3))
        sl = slice(m, lmax + 1)
        out[0].append(np.sqrt(tt[sl]) * g1)
        out[1].append(c_te[sl] * g1 + c_ee[sl] * g2)
        out[2].append(np.sqrt(bb[sl]) * g3)
    return np.stack([np.concatenate(o) for o in out])


def pol_noise_model(sigma2_t, p_factor=2.0, qu_corr_max=0.3, model_seed=0):
    """Per-pixel 3x3 noise covariance: T variance sigma2_t, Q and U variance
    p_factor sigma2_t with a Q-U correlation coefficient drawn uniformly in
    [-qu_corr_max, qu_corr_max] per pixel (stream 5 of model_seed); T uncorrelated with
    Q and U. Returns (cov6, ninv6), each [6, npix] in the order TT, QQ, UU, TQ, TU, QU;
    ninv6 is the inverse of the covariance (the QU block inverted in closed form)."""
    s2 = np.asarray(sigma2_t, dtype=np.float64)
    rho = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(model_seed), 5]))).uniform(
        -qu_corr_max, qu_corr_max, s2.size)
    sp = p_factor * s2
    z = np.zeros_like(s2)
    cov6 = np.stack([s2, sp, sp, z, z, rho * sp])
    det = sp * sp * (1.0 - rho * rho)
    ninv6 = np.stack([1.0 / s2, sp / det, sp / det, z, z, -rho * sp / det])
    return cov6, ninv6


def pol_noise_draw(cov6, seed):
    """Noise maps [3, npix] with the per-pixel covariance cov6 (Cholesky of each 3x3
    block), from the noise stream of `seed`; drawn everywhere, also where masked."""
    tt, qq, uu, tq, tu, qu = np.asarray(cov6, dtype=np.float64)
    g = rng(seed, 1).standard_normal((3, tt.size))
    l00 = np.sqrt(tt)
    l10 = tq / l00
    l20 = tu / l00
    l11 = np.sqrt(qq - l10 * l10)
    l21 = (qu - l20 * l10) / l11
    l22 = np.sqrt(uu - l20 * l20 - l21 * l21)
    return np.stack([l00 * g[0], l10 * g[0] + l11 * g[1], l20 * g[0] + l21 * g[1] + l22 * g[2]])


def pol_mask_bits(mask_t, mask_p):
    """Mask bytes: bit 0 set where T is observed, bit 1 where Q/U are (True = masked in)."""
    return ((~np.asarray(mask_t)).astype(np.uint8) | ((~np.asarray(mask_p)).astype(np.uint8) << 1))


def pol_small_case(theta, lmax, seed=0, model_seed=0):
    """Small polarised case (Nside 4..64 tests): TT = 1e3/(l(l+1)), cl_pol defaults;
    T noise (30 muK)^2 / h_p as in the small band case, P noise twice that with Q-U
    correlations; T mask |theta - pi/2| < 0.35 rad, P mask |theta - pi/2| < 0.5 rad."""
    lmax = int(lmax)
    cl4 = cl_pol(cl_power_law(lmax))
    h = np.exp(0.5 * rng(model_seed, 2).standard_normal(theta.size))
    cov6, ninv6 = pol_noise_model((30.0 * MUK) ** 2 / h, model_seed=model_seed)
    mask_t = np.abs(theta - 0.5 * np.pi) < 0.35
    mask_p = np.abs(theta - 0.5 * np.pi) < 0.5
    return {"cl4": cl4, "cov6": cov6, "ninv6": ninv6, "mask": pol_mask_bits(mask_t, mask_p),
            "mask_t": mask_t, "mask_p": mask_p, "lmax": lmax,
            "signal_alm": random_alm_pol(cl4, lmax, seed), "noise": pol_noise_draw(cov6, seed),
            "schedule": geometric_schedule(1e4, 40, 100)}


def pol_satellite_case(theta, phi, lmax, seed=0, model_seed=0, nobs_scale=1.0, pcut_deg=20.0, **kw):
    """Satellite-style polarised case: the temperature recipe of `satellite_model` (its
    spectrum, N_obs noise and |b| < 15 deg + discs mask) for T; cl_pol spectra; P noise
    twice the T variance with Q-U correlations; P mask |b| < pcut_deg plus the same discs."""
    t = satellite_model(theta, phi, lmax, model_seed=model_seed, nobs_scale=nobs_scale, **kw)
    cl4 = cl_pol(t["cl"])
    cov6, ninv6 = pol_noise_model(t["sigma2"], model_seed=model_seed)
    mask_p = t["mask"] | galactic_cut(theta, pcut_deg)
    return {"cl4": cl4, "cov6": cov6, "ninv6": ninv6, "mask": pol_mask_bits(t["mask"], mask_p),
            "mask_t": t["mask"], "mask_p": mask_p, "lmax": int(lmax), "schedule": t["schedule"],
            "signal_alm": random_alm_pol(cl4, lmax, seed), "noise": pol_noise_draw(cov6, seed)}
