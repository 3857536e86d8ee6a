"""Synthetic stand-ins for the paper's workloads (its datasets are not
available): color images, old-video-shaped clips and multispectral cubes with
values in [0, 1] (Section 4 normalizes every dataset to [0, 1]), Bernoulli
sampling masks at the paper's sampling rates, and N(0, 1) initial factors
(Algorithm 1, initialization).

Every draw uses NumPy's PCG64 seeded through a SeedSequence; data, mask and
initial factors come from three independent child streams of one seed.
"""

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# bookkeeping shared by both sides (shapes only, no arithmetic of the method)
# ----------------------------------------------------------------------------

def _pairs(N):
    return [(i, j) for i in range(N) for j in range(i + 1, N)]


def factor_shapes_of(dims, ranks):
    """Factor k has modes (R_1k, .., R_{k-1,k}, I_k, R_{k,k+1}, .., R_kN); the
    rank vector is ordered R_12, R_13, .., R_1N, R_23, .., R_{N-1,N}."""
    N = len(dims)
    R = [[0] * N for _ in range(N)]
    pairs = _pairs(N)
    if len(ranks) != len(pairs):
        raise ValueError("rank vector length must be N(N-1)/2")
    for (i, j), r in zip(pairs, ranks):
        R[i][j] = R[j][i] = int(r)
    return [tuple(dims[k] if j == k else R[k][j] for j in range(N)) for k in range(N)]


def _streams(seed):
    ss = np.random.SeedSequence(seed)
    data, mask, init = ss.spawn(3)
    return (np.random.Generator(np.random.PCG64(data)),
            np.random.Generator(np.random.PCG64(mask)),
            np.random.Generator(np.random.PCG64(init)))


def init_factors(rng, dims, ranks):
    """N(0, 1) float64 initial factors (Algorithm 1: rand(.) is standard normal)."""
    return [rng.standard_normal(s) for s in factor_shapes_of(dims, ranks)]


def rank_growth_draws(seed, dims):
    """Draws for the rank-increasing schedule: fill(g, ranks) returns N(0, 1)
    float64 arrays with the factor shapes at `ranks`, from a PCG64 stream keyed
    by (seed, g), so both sides of a comparison see the same values."""
    def fill(g, ranks):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77, g])))
        return [rng.standard_normal(s) for s in factor_shapes_of(dims, ranks)]
    return fill


def seeded_normal_factors(seed, dims, ranks):
    """The initial factors the library draws from a seed when a plan is made
    without host factors: a counter-based SplitMix64 stream (Steele, Lea and
    Flood, OOPSLA 2014; word j = mix(seed + (j + 1) * 0x9E3779B97F4A7C15)),
    pairs of words turned into pairs of standard normals by the Box-Muller
    transform (u1 = ((w >> 11) + 1) 2^-53 in (0, 1], u2 = (w >> 11) 2^-53;
    sqrt(-2 ln u1) cos(2 pi u2), then sin), factor 1's entries first.  The
    library implements the same published definition independently."""
    M = (1 << 64) - 1
    gamma = 0x9E3779B97F4A7C15

    def words(j):
        z = (seed + (j + 1) * gamma) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    shapes = factor_shapes_of(dims, ranks)
    total = sum(int(np.prod(sh)) for sh in shapes)
    npairs = (total + 1) // 2
    w = np.array([words(j) for j in range(2 * npairs)], dtype=np.uint64)
    u1 = ((w[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npairs)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    out, off = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(z[off:off + n].reshape(sh).copy())
        off += n
    return out


def bernoulli_mask(rng, shape, sr):
    """Omega: each entry observed independently with probability sr (uint8)."""
    return (rng.random(shape) < sr).astype(np.uint8)


# ----------------------------------------------------------------------------
# ground-truth generators
# ----------------------------------------------------------------------------

def lowrank_order3(rng, dims, rank=3, taps=5):
    """Order-3 low-FCTN-rank tensor: Gaussian factors with all bonds `rank`,
    each circularly box-filtered (`taps` taps) along its physical mode, then
    combined by the FCTN sum over the three bonds and min-max scaled to [0, 1].
    The single einsum below is data synthesis, written independently of both
    the oracle and the GPU library."""
    I1, I2, I3 = dims
    shapes = factor_shapes_of(dims, (rank, rank, rank))
    fs = []
    for k, s in enumerate(shapes):
        a = rng.standard_normal(s)
        acc = np.zeros_like(a)
        for d in range(-(taps // 2), taps // 2 + 1):
            acc += np.roll(a, d, axis=k)
        fs.append(acc / taps)
    x = np.einsum("iab,ajc,bck->ijk", fs[0], fs[1], fs[2])
    return (x - x.min()) / (x.max() - x.min())


def lowrank_order5(rng, dims, rank=3, taps=5):
    """Order-5 low-FCTN-rank tensor built like lowrank_order3: Gaussian factors
    with all ten bonds `rank`, each circularly box-filtered along its physical
    mode, combined by the FCTN sum over the ten bonds (one einsum, data
    synthesis only) and min-max scaled to [0, 1]."""
    shapes = factor_shapes_of(dims, (rank,) * 10)
    fs = []
    for k, s in enumerate(shapes):
        a = rng.standard_normal(s)
        acc = np.zeros_like(a)
        for d in range(-(taps // 2), taps // 2 + 1):
            acc += np.roll(a, d, axis=k)
        fs.append(acc / taps)
    x = np.einsum("iABCD,AjEFG,BEkHI,CFHlJ,DGIJm->ijklm", *fs, optimize="greedy")
    return (x - x.min()) / (x.max() - x.min())


def color_image(rng, H, W, n_sines=8, n_ellipses=6):
    """H x W x 3 color image in [0, 1]: per channel 0.5 plus n_sines random 2-D
    sinusoids (amplitude U(0.02, 0.1), frequency U(0.5, 8) cycles per image
    along each axis with a random sign, phase U(0, 2 pi)), then n_ellipses
    constant-valued ellipses (value U(0, 1), center U(0.1, 0.9), semi-axes
    U(0.05, 0.25), angle U(0, pi)) painted over; channels mixed by a random
    row-stochastic 3 x 3 matrix; clipped to [0, 1]."""
    y, x = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    chans = []
    for _ in range(3):
        img = np.full((H, W), 0.5)
        for _ in range(n_sines):
            amp = rng.uniform(0.02, 0.1)
            fx = rng.uniform(0.5, 8.0) * rng.choice([-1.0, 1.0])
            fy = rng.uniform(0.5, 8.0) * rng.choice([-1.0, 1.0])
            ph = rng.uniform(0.0, 2 * np.pi)
            img += amp * np.sin(2 * np.pi * (fx * x + fy * y) + ph)
        for _ in range(n_ellipses):
            val = rng.uniform(0.0, 1.0)
            cy, cx = rng.uniform(0.1, 0.9, size=2)
            ay, ax = rng.uniform(0.05, 0.25, size=2)
            th = rng.uniform(0.0, np.pi)
            dy, dx = y - cy, x - cx
            u = dx * np.cos(th) + dy * np.sin(th)
            v = -dx * np.sin(th) + dy * np.cos(th)
            img[(u / ax) ** 2 + (v / ay) ** 2 <= 1.0] = val
        chans.append(img)
    img = np.stack(chans, axis=-1)
    mix = rng.uniform(0.0, 1.0, size=(3, 3))
    mix /= mix.sum(axis=1, keepdims=True)
    return np.clip(img @ mix.T, 0.0, 1.0)


def _shift_periodic(img, dy, dx):
    """Periodic bilinear resample of img (H x W x C) shifted by (dy, dx) px."""
    iy, fy = int(np.floor(dy)), dy - np.floor(dy)
    ix, fx = int(np.floor(dx)), dx - np.floor(dx)
    a = np.roll(img, (iy, ix), axis=(0, 1))
    b = np.roll(img, (iy + 1, ix), axis=(0, 1))
    c = np.roll(img, (iy, ix + 1), axis=(0, 1))
    d = np.roll(img, (iy + 1, ix + 1), axis=(0, 1))
    return ((1 - fy) * (1 - fx) * a + fy * (1 - fx) * b
            + (1 - fy) * fx * c + fy * fx * d)


def video(rng, H, W, T, noise=0.01):
    """H x W x 3 x T clip: frame 0 is color_image(H, W); frame t is frame 0
    shifted by the cumulative drift sum_{tau <= t} d_tau with d_tau ~ U(-1, 1)^2
    px (periodic bilinear), plus N(0, noise^2) noise, clipped to [0, 1]."""
    f0 = color_image(rng, H, W)
    out = np.empty((H, W, 3, T))
    drift = np.zeros(2)
    for t in range(T):
        if t > 0:
            drift += rng.uniform(-1.0, 1.0, size=2)
        fr = _shift_periodic(f0, drift[0], drift[1])
        fr = fr + rng.normal(0.0, noise, size=fr.shape)
        out[:, :, :, t] = np.clip(fr, 0.0, 1.0)
    return out


def multispectral(rng, H, W, B=31, n_end=8, n_peaks=4):
    """H x W x B cube: sum over n_end endmembers of a smooth Gaussian-blob
    abundance map (center U(0.1, 0.9), sigma U(0.05, 0.3) of the side) times a
    spectrum of n_peaks Gaussian peaks on a B-point 400-700 nm grid (center
    U(400, 700), width U(15, 60) nm, amplitude U(0.2, 1)); min-max to [0, 1]."""
    y, x = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    lam = np.linspace(400.0, 700.0, B)
    cube = np.zeros((H, W, B))
    for _ in range(n_end):
        cy, cx = rng.uniform(0.1, 0.9, size=2)
        sg = rng.uniform(0.05, 0.3)
        ab = np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * sg * sg))
        spec = np.zeros(B)
        for _ in range(n_peaks):
            c = rng.uniform(400.0, 700.0)
            w = rng.uniform(15.0, 60.0)
            a = rng.uniform(0.2, 1.0)
            spec += a * np.exp(-((lam - c) ** 2) / (2 * w * w))
        cube += ab[:, :, None] * spec[None, None, :]
    return (cube - cube.min()) / (cube.max() - cube.min())


def multitemporal(rng, H, W, B=4, T=5, n_end=6, n_peaks=3):
    """H x W x B x T multi-temporal cube (height, width, band, time): n_end
    endmembers, each a spectrum of n_peaks Gaussian peaks sampled at B band
    centres spread over 450-850 nm (peak centre U(450, 850), width U(40, 150)
    nm, amplitude U(0.2, 1)) times a Gaussian-blob abundance map (centre
    U(0.1, 0.9), sigma U(0.05, 0.3) of the side); between acquisitions each
    blob centre drifts by U(-0.02, 0.02) of the side and its amplitude follows
    1 + 0.3 sin(2 pi t / T + phase), phase U(0, 2 pi); min-max to [0, 1]."""
    y, x = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    lam = np.linspace(450.0, 850.0, B)
    cube = np.zeros((H, W, B, T))
    for _ in range(n_end):
        cy, cx = rng.uniform(0.1, 0.9, size=2)
        sg = rng.uniform(0.05, 0.3)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        spec = np.zeros(B)
        for _ in range(n_peaks):
            c = rng.uniform(450.0, 850.0)
            w = rng.uniform(40.0, 150.0)
            a = rng.uniform(0.2, 1.0)
            spec += a * np.exp(-((lam - c) ** 2) / (2 * w * w))
        for t in range(T):
            if t > 0:
                cy, cx = np.array([cy, cx]) + rng.uniform(-0.02, 0.02, size=2)
            amp = 1.0 + 0.3 * np.sin(2.0 * np.pi * t / T + phase)
            ab = amp * np.exp(-((y - cy) ** 2 + (x - cx) ** 2) / (2 * sg * sg))
            cube[:, :, :, t] += ab[:, :, None] * spec[None, None, :]
    return (cube - cube.min()) / (cube.max() - cube.min())


# ----------------------------------------------------------------------------
# problem configurations
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    dims: tuple
    ranks: tuple
    truth: np.ndarray          # ground truth in the storage dtype
    Y: np.ndarray              # observed tensor (zero off Omega), storage dtype
    mask: np.ndarray           # uint8, nonzero = observed
    A0: list                   # float64 initial factors
    lam: float = 1e-2
    delta: float = 0.5
    rho: float = 0.1
    sweeps: int = 50
    precision: str = "f32"
    sr: float = 0.1
    extra: dict = field(default_factory=dict)


# name -> (kind, dims, ranks, sr, sweeps, precision)
CONFIGS = {
    "c1": ("lowrank3", (32, 32, 8), (3, 3, 3), 0.3, 50, "f64"),
    "c2": ("image", (256, 256, 3), (12, 3, 3), 0.1, 100, "f32"),
    "c3": ("video", (144, 176, 3, 50), (8, 3, 8, 3, 8, 3), 0.05, 100, "f32"),
    "c4": ("spectral", (512, 512, 31), (16, 8, 8), 0.05, 80, "bf16"),
    # the paper's second workload set, at its own shapes (Section 4): a new
    # color video (500 x 550 x 3 x 24) and a multi-temporal multispectral
    # image (300 x 300 x 4 bands x 5 dates)
    "c5": ("video", (500, 550, 3, 24), (8, 3, 8, 3, 8, 3), 0.05, 100, "f32"),
    "c6": ("multitemporal", (300, 300, 4, 5), (8, 3, 4, 3, 4, 3), 0.05, 100, "f32"),
    # Table 2's N-th order case at N = 5 (the paper runs no order-5 data)
    "c7": ("lowrank5", (32, 32, 32, 32, 8), (3,) * 10, 0.1, 50, "f32"),
}


def _truth(kind, rng, dims):
    if kind == "lowrank3":
        return lowrank_order3(rng, dims)
    if kind == "image":
        return color_image(rng, dims[0], dims[1])
    if kind == "video":
        return video(rng, dims[0], dims[1], dims[3])
    if kind == "spectral":
        return multispectral(rng, dims[0], dims[1], dims[2])
    if kind == "lowrank5":
        return lowrank_order5(rng, dims)
    if kind == "multitemporal":
        return multitemporal(rng, dims[0], dims[1], dims[2], dims[3])
    raise ValueError(kind)


def make_problem(name, seed=0, dims=None, ranks=None, sr=None, sweeps=None,
                 precision=None):
    """Build one configuration.  `dims` etc. override the named config (the
    generator of the named kind is kept), which gives reduced-size parity
    cases with the same structure."""
    kind, d0, r0, sr0, sw0, p0 = CONFIGS[name]
    dims = tuple(dims or d0)
    ranks = tuple(ranks or r0)
    sr = sr0 if sr is None else sr
    sweeps = sw0 if sweeps is None else sweeps
    precision = precision or p0
    rd, rm, ri = _streams(seed)
    truth = _truth(kind, rd, dims)
    store = np.float64 if precision == "f64" else np.float32
    truth = truth.astype(store)
    mask = bernoulli_mask(rm, dims, sr)
    Y = np.where(mask != 0, truth, 0).astype(store)
    A0 = init_factors(ri, dims, ranks)
    return Problem(name, dims, ranks, truth, Y, mask, A0, sweeps=sweeps,
                   precision=precision, sr=sr)


def serving_requests(seed=0, n=256, rate=20.0, sweeps=30):
    """Request mix: n requests with exponential inter-arrival times at `rate`
    per second; each draws uniformly one of six shape classes (order 3
    {64, 128, 256}^2 x 3 image-like with ranks (12, 3, 3); order 4
    72 x 88 x 3 x {10, 25, 50} video-like with ranks (8, 3, 8, 3, 8, 3)) and a
    sampling rate from {0.05, 0.1, 0.2}.  Returns a list of dicts with the
    arrival time and the generator arguments; the tensors are built lazily by
    make_problem with the request's own seed."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 5])))
    classes = [("c2", (64, 64, 3)), ("c2", (128, 128, 3)), ("c2", (256, 256, 3)),
               ("c3", (72, 88, 3, 10)), ("c3", (72, 88, 3, 25)), ("c3", (72, 88, 3, 50))]
    t = 0.0
    reqs = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        cname, dims = classes[int(rng.integers(len(classes)))]
        sr = float(rng.choice([0.05, 0.1, 0.2]))
        reqs.append({"id": i, "arrival": t, "config": cname, "dims": dims,
                     "sr": sr, "sweeps": sweeps, "seed": 1000 + i})
    return reqs
