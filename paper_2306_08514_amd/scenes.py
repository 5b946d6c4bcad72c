"""Seeded synthetic inputs: array geometries, candidate grids and multichannel
STFT frames.

This module generates the inputs of the SRP-map hot path and holds none of
its arithmetic (no cross-spectra, steering, sampling or interpolation).  Both
the HIP path and the FP64 oracle consume what it produces.

The paper evaluates on speech, babble noise and simulated or measured room
impulse responses (Sec. V), none of which ship here.  The scenes below are
synthetic stand-ins with the paper's structure: a band-limited coloured
source, free-field or image-source propagation with exact fractional delays
and 1/(4 pi r) spreading, sensor or diffuse noise at a stated SNR, and an
STFT with hop N/2 (Sec. V-B1).

All randomness comes from numpy.random.default_rng(2306085140 + index) in a
fixed draw order, so every consumer sees bit-identical frames.
"""

import numpy as np

SEED_BASE = 2306085140
C_SOUND = 343.0


# --------------------------------------------------------------- geometry --

def uca(M, diameter, center=(0.0, 0.0, 0.0)):
    """Uniform circular array in a horizontal plane, quoted by diameter."""
    a = 2.0 * np.pi * np.arange(M) / M
    c = np.asarray(center, dtype=np.float64)
    return np.stack([c[0] + diameter / 2 * np.cos(a),
                     c[1] + diameter / 2 * np.sin(a),
                     np.full(M, c[2])], axis=1)


def square_array(half=0.1):
    """Four microphones on a square in the plane z = 0, in the order
    (-,-), (+,-), (+,+), (-,+)."""
    return np.array([[-half, -half, 0.0], [half, -half, 0.0],
                     [half, half, 0.0], [-half, half, 0.0]])


def random_disc_array(rng, M, radius, z, min_spacing):
    """M microphones uniform in a horizontal disc, rejection-sampled so that
    no two are closer than min_spacing."""
    pts = []
    while len(pts) < M:
        r = radius * np.sqrt(rng.uniform())
        a = rng.uniform(0, 2 * np.pi)
        p = np.array([r * np.cos(a), r * np.sin(a), z])
        if all(np.linalg.norm(p - q) >= min_spacing for q in pts):
            pts.append(p)
    return np.array(pts)


def box_grid(xs, ys, zs):
    """Cartesian candidate grid, x-major, z-minor (inclusive linspaces)."""
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def half_sphere_directions(step_deg=2.0):
    """Far-field candidate directions (unit vectors from the array towards
    the source) on the lower half sphere z <= 0 at step_deg resolution in
    azimuth and elevation: rings at depression 0, step, ..., < 90 degrees,
    azimuth-minor, followed by the nadir.  2 degrees gives 45 x 180 + 1 =
    8,101 directions."""
    el = np.deg2rad(np.arange(0.0, 90.0 - 1e-9, step_deg))
    az = np.deg2rad(np.arange(0.0, 360.0 - 1e-9, step_deg))
    E, A = np.meshgrid(el, az, indexing="ij")
    u = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), -np.sin(E)], axis=-1).reshape(-1, 3)
    return np.concatenate([u, [[0.0, 0.0, -1.0]]], axis=0)


# ---------------------------------------------------------------- signals --

def one_over_f_noise(rng, n, pole=0.95):
    """White Gaussian noise through the one-pole filter s[n] = a s[n-1] + w[n]."""
    w = rng.standard_normal(n)
    # closed-form IIR by FFT-free recursion in blocks would be faster; lfilter
    # from scipy is fine and deterministic
    from scipy.signal import lfilter
    return lfilter([1.0], [1.0, -pole], w)


def _delay_sum(spec, nfft, delays, gains):
    """Sum of delayed, scaled copies of a signal given by its rfft spectrum:
    sum_i g_i s(t - tau_i), delays in samples, by a phase shift."""
    w = 2.0 * np.pi * np.arange(nfft // 2 + 1) / nfft
    acc = np.zeros_like(spec)
    for d, g in zip(delays, gains):
        acc += g * np.exp(-1j * w * d)
    return np.fft.irfft(spec * acc, n=nfft)


def image_sources(src, room, max_order, beta):
    """Image sources of a shoebox [0, room] up to total reflection order
    max_order, each with amplitude beta^(reflections)."""
    out = []
    opts = []
    for ax in range(3):
        L = room[ax]
        x = src[ax]
        # (coordinate, reflection count) for n in {-1, 0, 1}
        axis_opts = []
        for n in (-1, 0, 1):
            axis_opts.append((2 * n * L + x, abs(2 * n)))
            axis_opts.append((2 * n * L - x, abs(2 * n - 1)))
        opts.append([o for o in axis_opts if o[1] <= max_order])
    for ox in opts[0]:
        for oy in opts[1]:
            for oz in opts[2]:
                order = ox[1] + oy[1] + oz[1]
                if order <= max_order:
                    out.append((np.array([ox[0], oy[0], oz[0]]), beta ** order))
    return out


def stft_frames(x, N, hop, L):
    """STFT with a periodic Hann window of length N and the given hop.
    x: [M, T] real.  Returns complex128 [L, M, N/2 + 1]."""
    n = np.arange(N)
    win = 0.5 - 0.5 * np.cos(2.0 * np.pi * n / N)
    M = x.shape[0]
    out = np.empty((L, M, N // 2 + 1), dtype=np.complex128)
    for l in range(L):
        seg = x[:, l * hop:l * hop + N] * win[None, :]
        out[l] = np.fft.rfft(seg, axis=1)
    return out


def _scale_to_snr(sig, noise, snr_db):
    ps = np.mean(np.var(sig, axis=1))
    pn = np.mean(np.var(noise, axis=1))
    return noise * np.sqrt(ps / (pn * 10.0 ** (snr_db / 10.0)))


def render(rng, mics, sources, fs, T, snr_db, noise="white", room=None,
           max_order=0, beta=0.7, n_diffuse=64, c=C_SOUND):
    """Microphone signals [M, T] for independent 1/f sources at the given
    positions, with exact fractional delays, 1/(4 pi r) spreading, optional
    image sources, and white sensor or diffuse noise at snr_db."""
    M = mics.shape[0]
    paths = []
    for s in sources:
        if max_order > 0:
            paths.append(image_sources(s, room, max_order, beta))
        else:
            paths.append([(np.asarray(s, dtype=np.float64), 1.0)])
    maxdist = max(np.linalg.norm(p - m) for ps in paths for (p, _) in ps for m in mics)
    dmax = int(np.ceil(maxdist / c * fs)) + 2
    nfft = 1 << int(np.ceil(np.log2(T + dmax + 1)))
    sig = np.zeros((M, T))
    for ps in paths:
        spec = np.fft.rfft(one_over_f_noise(rng, nfft))
        for m in range(M):
            dl = [np.linalg.norm(p - mics[m]) / c * fs for (p, _) in ps]
            gl = [g / (4 * np.pi * np.linalg.norm(p - mics[m])) for (p, g) in ps]
            sig[m] = _delay_sum(spec, nfft, dl, gl)[dmax:dmax + T]
    if noise == "white":
        nz = rng.standard_normal((M, T))
    elif noise == "diffuse":
        # independent 1/f plane waves from directions uniform on the sphere
        v = rng.standard_normal((n_diffuse, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        nz_full = np.zeros((M, nfft // 2 + 1), dtype=np.complex128)
        w = 2.0 * np.pi * np.arange(nfft // 2 + 1) / nfft
        ctr = mics.mean(0)
        for i in range(n_diffuse):
            spec = np.fft.rfft(one_over_f_noise(rng, nfft))
            for m in range(M):
                # a plane wave arriving from direction v reaches a microphone
                # displaced towards v earlier
                d = -((mics[m] - ctr) @ v[i]) / c * fs + dmax / 2
                nz_full[m] += spec * np.exp(-1j * w * d)
        nz = np.fft.irfft(nz_full, n=nfft, axis=1)[:, dmax:dmax + T]
    else:
        raise ValueError(noise)
    return sig + _scale_to_snr(sig, nz, snr_db)


# -------------------------------------------------------------- workloads --

def _n_samples(L, N, hop):
    return (L - 1) * hop + N


WORKLOADS = ("square4_plane1k", "uca8_room125k", "disc32_box200k")
_SEED_OFFSET = {"square4_plane1k": 0, "uca8_room125k": 1, "disc32_box200k": 3}


def workload(name, L=None, grid_stride=1):
    """Geometry and sizes of the named workloads:

    square4_plane1k: M = 4 square (0.2 m) in z = 0; planar 32 x 32 grid over
       [-2, 2]^2 (J = 1024); fs 16 kHz, N = 512, L = 100; one free-field
       source in the plane at >= 0.5 m from the centre; white sensor noise
       at 10 dB.  (Also the inputs of the precision sweep.)
    uca8_room125k: M = 8 UCA, diameter 0.3 m, ceiling-mounted at
       (2.5, 2.5, 2.4) in a 5 x 5 x 2.5 m room; 50 x 50 x 50 grid over the
       room (J = 125,000); fs 16 kHz, N = 1024, L = 1000; one source >= 0.5 m
       from walls and array, z <= 2.0; image sources of order <= 2 with wall
       reflection 0.7; diffuse 1/f noise at 5 dB.
    disc32_box200k: M = 32 uniform in a disc of radius 1 m at z = 3.0
       (>= 5 cm spacing); 100 x 100 x 20 grid over [-5, 5]^2 x [0.5, 2.5]
       (J = 200,000); fs 48 kHz, N = 2048, L = 256; two free-field sources
       in the grid box; white sensor noise at 10 dB.

    Returns a dict with mics, grid, fs, N, hop, L, c and the drawing recipe;
    frames are produced by make_frames().  grid_stride subsamples every grid
    axis (for small test cases)."""
    if name not in _SEED_OFFSET:
        raise ValueError(f"no workload {name!r}; known: {WORKLOADS}")
    rng = np.random.default_rng(SEED_BASE + _SEED_OFFSET[name])
    if name == "square4_plane1k":
        mics = square_array(0.1)
        g = np.linspace(-2.0, 2.0, 32)[::grid_stride]
        grid = box_grid(g, g, np.array([0.0]))
        while True:
            s = np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), 0.0])
            if np.linalg.norm(s) >= 0.5:
                break
        cfg = dict(mics=mics, grid=grid, fs=16000.0, N=512, hop=256, L=L or 100,
                   sources=[s], snr_db=10.0, noise="white", room=None, max_order=0)
    elif name == "uca8_room125k":
        mics = uca(8, 0.3, (2.5, 2.5, 2.4))
        gx = np.linspace(0.0, 5.0, 50)[::grid_stride]
        gz = np.linspace(0.0, 2.5, 50)[::grid_stride]
        grid = box_grid(gx, gx, gz)
        room = np.array([5.0, 5.0, 2.5])
        while True:
            s = rng.uniform([0.5, 0.5, 0.5], [4.5, 4.5, 2.0])
            if np.min(np.linalg.norm(mics - s, axis=1)) >= 0.5:
                break
        cfg = dict(mics=mics, grid=grid, fs=16000.0, N=1024, hop=512, L=L or 1000,
                   sources=[s], snr_db=5.0, noise="diffuse", room=room, max_order=2)
    else:
        mics = random_disc_array(rng, 32, 1.0, 3.0, 0.05)
        gx = np.linspace(-5.0, 5.0, 100)[::grid_stride]
        gz = np.linspace(0.5, 2.5, 20)[::grid_stride]
        grid = box_grid(gx, gx, gz)
        srcs = [rng.uniform([-5, -5, 0.5], [5, 5, 2.5]) for _ in range(2)]
        cfg = dict(mics=mics, grid=grid, fs=48000.0, N=2048, hop=1024, L=L or 256,
                   sources=srcs, snr_db=10.0, noise="white", room=None, max_order=0)
    cfg["c"] = C_SOUND
    cfg["name"] = name
    cfg["_rng"] = rng
    return cfg


def make_frames(cfg):
    """Render the workload's signals and return complex64 STFT frames
    [L, M, N/2 + 1] (computed in FP64, then rounded once)."""
    rng = cfg["_rng"]
    T = _n_samples(cfg["L"], cfg["N"], cfg["hop"])
    x = render(rng, cfg["mics"], cfg["sources"], cfg["fs"], T, cfg["snr_db"],
               noise=cfg["noise"], room=cfg["room"], max_order=cfg["max_order"],
               c=cfg["c"])
    return stft_frames(x, cfg["N"], cfg["hop"], cfg["L"]).astype(np.complex64)


def random_frames(seed, L, M, N, zero_fraction=0.0):
    """Unstructured complex64 frames [L, M, N/2 + 1] (unit-variance complex
    Gaussian), optionally with a fraction of exact zeros, for edge-case
    tests."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    Y = (rng.standard_normal((L, M, N // 2 + 1)) + 1j * rng.standard_normal((L, M, N // 2 + 1)))
    if zero_fraction > 0:
        Y[rng.uniform(size=Y.shape) < zero_fraction] = 0.0
    return Y.astype(np.complex64)


# ------------------------------------------------------- evaluation scenes --

def evaluation_scene(kind, n_sources=16, frames_per_source=8, snr_db=12.0, max_order=0, beta=0.7,
                     grid_stride=2, seed=0):
    """Seeded scenes for the localisation and map-error sweeps, one source
    position per group of frames_per_source consecutive frames.

    room: the uca8_room125k array and grid (axes subsampled by grid_stride);
      sources uniform in the room >= 0.5 m from walls and array, z <= 2 m;
      image sources up to max_order (reflection beta); white noise at snr_db.
    square: the square4_plane1k array and 32 x 32 plane; sources in the
      plane >= 0.5 m from the centre.
    farfield: 8-mic UCA (0.3 m) at the origin, the 2-degree lower
      half-sphere of directions; 1/f plane waves (sources 300 m away) from
      uniformly drawn grid directions of depression 5..85 degrees.
    nf4: the paper's near-field scenario (Sec. V-B1, Table 1): M = 4
      microphones near the corners of a 4.9 x 5.9 x 3.5 m room at 3 m
      height, a 4 x 5 x 0.1 m grid at 3.33 cm around 1.5 m height (121 x
      151 x 4, J = 73,084), fs 4 kHz, 2K = 512, c = 340 m/s; sources
      uniform inside the grid volume.
    ff6: the paper's far-field scenario: a 6-mic UCA (diameter 0.3 m) 10 cm
      below the ceiling of a 6.5 x 9 x 4.5 m room, the 2-degree lower
      half-sphere (J = 8,101), fs 16 kHz, 2K = 1024, c = 340 m/s; sources
      inside the room at least 2 m from the array centre, their directions
      the truth.

    Returns (cfg, frames [n_sources * frames_per_source, M, N/2 + 1]
    complex64, truth [n_sources * frames_per_source, 3]) where truth holds
    source positions (room, square) or unit directions (farfield)."""
    rng = np.random.default_rng(SEED_BASE + 200 + seed)
    if kind == "room":
        cfg = workload("uca8_room125k", L=frames_per_source, grid_stride=grid_stride)
        room = np.array([5.0, 5.0, 2.5])
        far = False
    elif kind == "square":
        cfg = workload("square4_plane1k", L=frames_per_source)
        room, far = None, False
    elif kind == "farfield":
        cfg = dict(mics=uca(8, 0.3), grid=half_sphere_directions(2.0), fs=16000.0, N=1024, hop=512,
                   L=frames_per_source, c=C_SOUND, name="uca8_farfield8k")
        room, far = None, True
    elif kind == "nf4":
        mics = np.array([[0.4, 0.4, 3.0], [0.4, 5.4, 3.0], [4.4, 5.4, 3.0], [4.4, 0.4, 3.0]])
        grid = box_grid(np.linspace(0.4, 4.4, 121), np.linspace(0.4, 5.4, 151), np.linspace(1.45, 1.55, 4))
        cfg = dict(mics=mics, grid=grid, fs=4000.0, N=512, hop=256, L=frames_per_source, c=340.0,
                   name="nf4_paper73k")
        room, far = np.array([4.9, 5.9, 3.5]), False
    elif kind == "ff6":
        centre = np.array([3.25, 4.5, 4.4])
        cfg = dict(mics=uca(6, 0.3, centre), grid=half_sphere_directions(2.0), fs=16000.0, N=1024, hop=512,
                   L=frames_per_source, c=340.0, name="ff6_paper8k")
        room, far = np.array([6.5, 9.0, 4.5]), True
    else:
        raise ValueError(kind)
    N, hop = cfg["N"], cfg["hop"]
    T = _n_samples(frames_per_source, N, hop)
    frames, truth = [], []
    for _ in range(n_sources):
        if kind == "room":
            while True:
                s = rng.uniform([0.5, 0.5, 0.5], [4.5, 4.5, 2.0])
                if np.min(np.linalg.norm(cfg["mics"] - s, axis=1)) >= 0.5:
                    break
            src, t = s, s
        elif kind == "square":
            while True:
                s = np.array([rng.uniform(-2, 2), rng.uniform(-2, 2), 0.0])
                if np.linalg.norm(s) >= 0.5:
                    break
            src, t = s, s
        elif kind == "nf4":
            s = rng.uniform([0.4, 0.4, 1.45], [4.4, 5.4, 1.55])
            src, t = s, s
        elif kind == "ff6":
            ctr = cfg["mics"].mean(0)
            while True:
                s = rng.uniform([0.3, 0.3, 0.3], [6.2, 8.7, 4.0])
                if np.linalg.norm(s - ctr) >= 2.0:
                    break
            src, t = s, (s - ctr) / np.linalg.norm(s - ctr)
        else:
            g = cfg["grid"]
            dep = np.degrees(np.arcsin(-g[:, 2]))
            cand = np.nonzero((dep >= 5.0) & (dep <= 85.0))[0]
            t = g[cand[rng.integers(len(cand))]]
            src = 300.0 * t
        x = render(rng, cfg["mics"], [src], cfg["fs"], T, snr_db, noise="white", room=room,
                   max_order=max_order if room is not None else 0, beta=beta, c=cfg["c"])
        frames.append(stft_frames(x, N, hop, frames_per_source))
        truth.append(np.repeat(np.asarray(t, dtype=np.float64)[None], frames_per_source, axis=0))
    cfg["far_field"] = far
    return cfg, np.concatenate(frames).astype(np.complex64), np.concatenate(truth)


# ------------------------------------------------------------ serving mix --

SERVING_M = (4, 8, 16, 32)
SERVING_J = (1024, 16384, 125000, 200000)


def serving_array(M):
    """Array and sampling of the serving mix for M microphones: M = 4 is the
    0.2 m square (16 kHz, N = 512), M = 8 the 0.3 m UCA (16 kHz, N = 1024),
    M = 16 a 0.5 m UCA (16 kHz, N = 1024), M = 32 the 2 m-aperture random
    disc array (48 kHz, N = 2048).  Arrays are centred at the origin in the
    plane z = 0."""
    if M == 4:
        return square_array(0.1), 16000.0, 512
    if M == 8:
        return uca(8, 0.3), 16000.0, 1024
    if M == 16:
        return uca(16, 0.5), 16000.0, 1024
    if M == 32:
        rng = np.random.default_rng(SEED_BASE + 3)
        return random_disc_array(rng, 32, 1.0, 0.0, 0.05), 48000.0, 2048
    raise ValueError(M)


def serving_grid(J):
    """Candidate grids of the serving mix, relative to an array at the origin
    in the plane z = 0: 1k = 32 x 32 and 16k = 128 x 128 points in the array
    plane (over 4 x 4 m and 8 x 8 m); 125k = 50^3 over 5 x 5 x 2.5 m and
    200k = 100 x 100 x 20 over 10 x 10 x 2 m, both entirely below the array
    (z in [-3, -0.5] and [-2.5, -0.5]) so that no point has a mirror twin."""
    if J == 1024:
        g = np.linspace(-2.0, 2.0, 32)
        return box_grid(g, g, np.array([0.0]))
    if J == 16384:
        g = np.linspace(-4.0, 4.0, 128)
        return box_grid(g, g, np.array([0.0]))
    if J == 125000:
        return box_grid(np.linspace(-2.5, 2.5, 50), np.linspace(-2.5, 2.5, 50), np.linspace(-3.0, -0.5, 50))
    if J == 200000:
        return box_grid(np.linspace(-5.0, 5.0, 100), np.linspace(-5.0, 5.0, 100), np.linspace(-2.5, -0.5, 20))
    raise ValueError(J)


def serving_frames(M, L=256):
    """A pool of L seeded STFT frames for the M-microphone serving array: one
    free-field 1/f source 2 m below the array plane plus white sensor noise at
    10 dB."""
    mics, fs, N = serving_array(M)
    rng = np.random.default_rng(SEED_BASE + 100 + M)
    src = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), -2.0])
    T = _n_samples(L, N, N // 2)
    x = render(rng, mics, [src], fs, T, 10.0, noise="white")
    return stft_frames(x, N, N // 2, L).astype(np.complex64)
