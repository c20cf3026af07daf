"""Seeded synthetic catalogues -- the only module shared by the GPU tests and the oracle tests.

It holds no pair-counting arithmetic: it only draws point positions, weights
and bin edges.  The paper's own inputs (BOSS randoms, periodic random boxes of
its Sect. 5) are not available here; these generators stand in for them with
the shapes and sizes of the workloads named below.

Workloads (sizes in Mpc/h):
  C1  periodic cube L=1000, 20,000 uniform points, 40 linear s bins over [0,200).
  C2  periodic cube L=2000, 1,000,000 lognormal points (256^3 Gaussian field,
      P(k) ~ k^-1.5, sigma_G=1), 40 s bins over [0,200) x 100 mu bins over [0,1],
      line of sight z, optional weights U[0.5,1.5).
  C3  open survey-like shell: r in [1000,2000] with density ~ r^2, RA in [0,60) deg,
      sin(Dec) uniform for Dec in [-15,15) deg; data 2,000,000, randoms 20x;
      40 s_perp x 40 pi bins over [0,200), mid-point line of sight, weights U[0.5,2).
  C4  200 periodic L=1000 lognormal mocks with sizes uniform in [100k,500k].
  C5  periodic L=3000, 10,000,000 lognormal points, 50 log s bins over [0.1,50).
"""
import numpy as np

GENERATOR_VERSION = 1
SEED_BASE = 2301125570          # config c uses SEED_BASE + c
MOCK_SEED_BASE = 23011255740000  # batched mock m uses MOCK_SEED_BASE + m


def config_seed(c):
    return SEED_BASE + int(c)


def _guard_box(x, L):
    """Keep every coordinate inside [0, L): u*L can round up to L."""
    np.minimum(x, np.nextafter(L, 0.0), out=x)
    np.maximum(x, 0.0, out=x)
    return x


def uniform_box(n, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.random((int(n), 3)) * float(L)
    return _guard_box(x, float(L))


def blobs_box(n, L, nblob, rad, frac, seed):
    """A catalogue far more clustered than a lognormal field: a fraction `frac`
    of the n points in nblob Gaussian blobs of width `rad` (centres at least
    3 rad from the faces), the rest uniform, in [0, L)^3."""
    rng = np.random.default_rng(seed)
    nb = int(n * frac)
    cen = rng.uniform(rad * 3, L - rad * 3, (nblob, 3))
    x = cen[rng.integers(0, nblob, nb)] + rng.normal(0, rad, (nb, 3))
    x = np.concatenate([x, rng.uniform(0, L, (n - nb, 3))])
    return np.clip(x, 0, np.nextafter(L, 0))


def gaussian_field(ngrid, L, slope, sigma, rng):
    """Gaussian random field on ngrid^3 cells with P(k) ~ k^slope (k=0 removed), unit->sigma variance."""
    g = rng.standard_normal((ngrid, ngrid, ngrid))
    gk = np.fft.rfftn(g)
    kf = 2.0 * np.pi / L
    kx = np.fft.fftfreq(ngrid, d=1.0 / ngrid) * kf
    kz = np.fft.rfftfreq(ngrid, d=1.0 / ngrid) * kf
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)   # sqrt(P) = k^(slope/2)
    gk *= amp
    G = np.fft.irfftn(gk, s=(ngrid, ngrid, ngrid), axes=(0, 1, 2))
    G -= G.mean()
    G *= sigma / G.std()
    return G


def lognormal_box(n, L, seed, ngrid=256, slope=-1.5, sigma=1.0):
    """Clustered points: density ~ exp(G - sigma^2/2) with G the field above.

    Per-cell counts are multinomial with total exactly n (Poisson sampling
    conditioned on n): n cell indices are drawn i.i.d. with probability
    proportional to the density, then each point is placed uniformly in its cell.
    """
    rng = np.random.default_rng(seed)
    L = float(L)
    G = gaussian_field(ngrid, L, slope, sigma, rng)
    rho = np.exp(G - 0.5 * sigma * sigma).ravel()
    cdf = np.cumsum(rho)
    u = rng.random(int(n)) * cdf[-1]
    idx = np.searchsorted(cdf, u, side="right")
    np.minimum(idx, ngrid ** 3 - 1, out=idx)
    iz = idx % ngrid
    iy = (idx // ngrid) % ngrid
    ix = idx // (ngrid * ngrid)
    cellsz = L / ngrid
    off = rng.random((int(n), 3))
    x = np.empty((int(n), 3))
    x[:, 0] = (ix + off[:, 0]) * cellsz
    x[:, 1] = (iy + off[:, 1]) * cellsz
    x[:, 2] = (iz + off[:, 2]) * cellsz
    return _guard_box(x, L)


def survey_shell(n, seed, rmin=1000.0, rmax=2000.0, ra_deg=60.0, dec_half_deg=15.0):
    """Uniform points in a shell patch seen from the origin (density ~ r^2 in r)."""
    rng = np.random.default_rng(seed)
    n = int(n)
    u = rng.random((n, 3))
    r = np.cbrt(rmin ** 3 + u[:, 0] * (rmax ** 3 - rmin ** 3))
    ra = np.deg2rad(ra_deg) * u[:, 1]
    s0 = np.sin(np.deg2rad(-dec_half_deg))
    s1 = np.sin(np.deg2rad(dec_half_deg))
    sdec = s0 + u[:, 2] * (s1 - s0)
    cdec = np.sqrt(np.maximum(0.0, 1.0 - sdec * sdec))
    x = np.empty((n, 3))
    x[:, 0] = r * cdec * np.cos(ra)
    x[:, 1] = r * cdec * np.sin(ra)
    x[:, 2] = r * sdec
    return x


def uniform_weights(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random(int(n))


def s2_samples(n, rmax, seed):
    """Squared separations with P(s) ~ s^2 on [0, rmax): s^2 = x^(2/3) rmax^2 (App. C)."""
    rng = np.random.default_rng(seed)
    return rng.random(int(n)) ** (2.0 / 3.0) * float(rmax) ** 2


def s2_samples_torch(n, rmax, seed, device="cuda"):
    """s2_samples drawn with torch's Philox generator on `device` (float64), for
    the benchmark sizes (6.4e9 values); generated in place, so the only memory
    is the 8 n bytes of the result.  A different stream of numbers from
    s2_samples for the same seed."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    v = torch.empty(int(n), dtype=torch.float64, device=device)
    step = 1 << 28
    for lo in range(0, int(n), step):
        part = v[lo:lo + step]
        part.uniform_(0.0, 1.0, generator=g)
        part.pow_(2.0 / 3.0).mul_(float(rmax) ** 2)
    return v


def linear_edges(lo, hi, n):
    return np.linspace(float(lo), float(hi), int(n) + 1)


def log_edges(lo, hi, n):
    """exp(log(lo) + k*step), endpoints set exactly to lo and hi."""
    e = np.exp(np.log(lo) + np.arange(int(n) + 1) * (np.log(hi) - np.log(lo)) / n)
    e[0] = lo
    e[-1] = hi
    return e


def mu_edges(n):
    """k/n exactly as float64, k = 0..n."""
    return np.arange(int(n) + 1, dtype=np.float64) / float(n)


# ---------------------------------------------------------------------------
# Workload descriptions (scale < 1 shrinks point counts for quick tests)
# ---------------------------------------------------------------------------

def workload(c, scale=1.0, weighted=False, seed=None):
    """Return a dict describing workload c (1..5) with its catalogue(s) drawn."""
    c = int(c)
    sd = config_seed(c) if seed is None else int(seed)
    if c == 1:
        n = max(2, int(round(20000 * scale)))
        x = uniform_box(n, 1000.0, sd)
        w = uniform_weights(n, 0.5, 1.5, sd + 7) if weighted else None
        return dict(name="C1", x1=x, w1=w, box=1000.0, kind="s", los="z",
                    edges1=linear_edges(0, 200, 40), edges2=None)
    if c == 2:
        n = max(2, int(round(1_000_000 * scale)))
        x = lognormal_box(n, 2000.0, sd)
        w = uniform_weights(n, 0.5, 1.5, sd + 7) if weighted else None
        return dict(name="C2", x1=x, w1=w, box=2000.0, kind="smu", los="z",
                    edges1=linear_edges(0, 200, 40), edges2=mu_edges(100))
    if c == 3:
        nd = max(2, int(round(2_000_000 * scale)))
        nr = 20 * nd
        d = survey_shell(nd, sd)
        r = survey_shell(nr, sd + 1)
        wd = uniform_weights(nd, 0.5, 2.0, sd + 7) if weighted else None
        wr = uniform_weights(nr, 0.5, 2.0, sd + 8) if weighted else None
        return dict(name="C3", x1=d, w1=wd, x2=r, w2=wr, box=0.0, kind="spi", los="mid",
                    edges1=linear_edges(0, 200, 40), edges2=linear_edges(0, 200, 40))
    if c == 5:
        n = max(2, int(round(10_000_000 * scale)))
        x = lognormal_box(n, 3000.0, sd)
        return dict(name="C5", x1=x, w1=None, box=3000.0, kind="s", los="z",
                    edges1=log_edges(0.1, 50.0, 50), edges2=None)
    raise ValueError(f"workload {c}: use mock_sizes/mock for the batched set")


def mock_sizes(nmock=200, lo=100_000, hi=500_000, seed=None, scale=1.0):
    rng = np.random.default_rng(config_seed(4) if seed is None else seed)
    sz = rng.integers(lo, hi + 1, size=int(nmock))
    return np.maximum(2, np.round(sz * scale).astype(np.int64))


def mock(m, n, L=1000.0, ngrid=256):
    return lognormal_box(int(n), L, MOCK_SEED_BASE + int(m), ngrid=ngrid)


def lognormal_box_torch(n, L, seed, device="cuda", ngrid=256, slope=-1.5, sigma=1.0):
    """The generator of lognormal_box with torch operations on `device` (float64),
    for producing many large mocks quickly.  Seeded with torch's Philox generator
    of that device, so its draws differ from the numpy version's."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    L = float(L)
    noise = torch.randn((ngrid, ngrid, ngrid), generator=g, device=device, dtype=torch.float64)
    gk = torch.fft.rfftn(noise)
    kf = 2.0 * torch.pi / L
    kx = torch.fft.fftfreq(ngrid, d=1.0 / ngrid, device=device, dtype=torch.float64) * kf
    kz = torch.fft.rfftfreq(ngrid, d=1.0 / ngrid, device=device, dtype=torch.float64) * kf
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (slope / 4.0), torch.zeros_like(k2))
    G = torch.fft.irfftn(gk * amp, s=(ngrid, ngrid, ngrid))
    G = (G - G.mean()) * (sigma / G.std())
    rho = torch.exp(G - 0.5 * sigma * sigma).reshape(-1)
    cdf = torch.cumsum(rho, 0)
    u = torch.rand(int(n), generator=g, device=device, dtype=torch.float64) * cdf[-1]
    idx = torch.searchsorted(cdf, u, right=True).clamp_max(ngrid ** 3 - 1)
    iz = idx % ngrid
    iy = (idx // ngrid) % ngrid
    ix = idx // (ngrid * ngrid)
    off = torch.rand((int(n), 3), generator=g, device=device, dtype=torch.float64)
    cell = L / ngrid
    x = torch.stack([(ix + off[:, 0]) * cell, (iy + off[:, 1]) * cell, (iz + off[:, 2]) * cell], dim=1)
    return x.clamp_(0.0, float(np.nextafter(L, 0.0))).contiguous()
