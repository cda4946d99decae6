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
