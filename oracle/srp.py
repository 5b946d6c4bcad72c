"""Plain FP64 numpy oracle of the SRP-map hot path (arXiv 2306.08514).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code,
tables or constants with the HIP library; the two meet only in the seeded
input generator, which holds none of the method's arithmetic.

Every function is written from the paper's definitions, in FP64, with numpy
primitives (FFT, SVD, sort, matrix products) as single steps and no blocking
or reordering beyond what the definition states (the only exception is
chunking over candidate locations to bound memory, which does not change the
arithmetic of any output element).

Equation numbers refer to the paper's numbered equations.  Readings of points
where the paper is silent or inconsistent:

* K is half the DFT length N = 2K; the bins used are k = 1..K-1 (Sec. II-D).
  The DC and Nyquist values of every cross-spectrum are taken as zero, which
  makes the single- and two-sided forms (Appendix) and the iFFT sampling (46)
  exact.
* The map keeps the factor 2 of (22); the iFFT is unnormalised, so that
  xi_p = 2 Re[S_p psi_p] (40) holds with the samples of (46).
* PHAT weighting (2) with psi = 0 wherever y_m y_m'^* = 0.
* sinc is the normalised sinc sin(pi t)/(pi t) of Whittaker-Shannon (31).
* Pairs are enumerated p <-> (m, m'), m > m', with m' in the outer and m in
  the inner loop, the summation order of (8).
* SLRI is taken per pair (rank R per pair, U_p (V_p^T xi_p)) as well as in the
  paper's global form; SSPI keeps the Q largest-magnitude entries per
  (location, pair) as well as the paper's global top-Q_Lambda.  Ties in the
  SSPI selection go to the smaller |x - n|, then the smaller n.
* Argmax ties go to the smallest location index.

Parity status: every function below is pinned by the CPU tests in
``tests/test_oracle_pins.py`` against values printed in the paper (Table 1,
Fig. 12, the measured-array layout), closed forms (integer-delay GCC, the
Dirichlet-kernel map of a single pure-delay source, the exact periodic
interpolator) and brute force (delay-and-sum output power).
``slri_factors_gram`` (the same truncation through the Gram matrix, for
very tall Lambda_p) is pinned against ``slri_factors``, which the
Eckart-Young and full-rank checks pin.  The far-field TDOA is pinned as the
far limit of the near-field model; LR-SRP by full rank (= conv. FD-SRP),
Eckart-Young optimality and its complexity (30) in Fig. 12.
"""

import numpy as np

__all__ = [
    "pairs", "tdoa_samples", "tdoa_samples_far_field", "max_lags",
    "mean_lags", "phat", "steering", "fd_map", "two_sided",
    "gcc_samples_ifft", "gcc_samples_direct", "interp_matrix", "si_map",
    "td_map", "slri_factors", "slri_factors_gram", "slri_map", "slri_global_factors",
    "slri_global_map", "sspi_select", "sspi_map", "sspi_global_select",
    "sspi_global_map", "dsb_power_map", "argmax_map", "rel_error",
    "eps_z_db", "eps_h_db", "complexity", "periodic_interp_map",
    "stack_samples", "steering_matrix", "lr_factors", "lr_map",
]


# --------------------------------------------------------------------------
# Geometry: pairs, TDOAs, lag ranges (Sec. II-A, Sec. III-B1)
# --------------------------------------------------------------------------

def pairs(M):
    """Microphone pairs p <-> (m, m') with m > m' (Sec. II-A), enumerated in
    the order of the double sum of (8): m' outer, m inner.  0-based."""
    return [(m, mp) for mp in range(M - 1) for m in range(mp + 1, M)]


def tdoa_samples(mics, grid, fs, c):
    """Near-field TDOA of every pair at every candidate, in samples:
    x_p(j) = (||r_m - q_j|| - ||r_m' - q_j||) fs / c, i.e. Delta t_p(j)/T with
    the near-field case of (3).  Returns an array of shape [P, J]."""
    mics = np.asarray(mics, dtype=np.float64)
    grid = np.asarray(grid, dtype=np.float64)
    dist = np.sqrt(((grid[None, :, :] - mics[:, None, :]) ** 2).sum(-1))  # [M, J]
    out = np.empty((len(pairs(len(mics))), grid.shape[0]), dtype=np.float64)
    for p, (m, mp) in enumerate(pairs(len(mics))):
        out[p] = (dist[m] - dist[mp]) * fs / c
    return out


def tdoa_samples_far_field(mics, directions, fs, c):
    """Far-field TDOA in samples for unit source directions u (pointing from
    the array towards the source).  This is the far limit of the near-field
    model, x_p = -(r_m - r_m')^T u fs / c; the paper's far-field case of (3)
    writes it with the incident (propagation) direction q = -u."""
    mics = np.asarray(mics, dtype=np.float64)
    u = np.asarray(directions, dtype=np.float64)
    out = np.empty((len(pairs(len(mics))), u.shape[0]), dtype=np.float64)
    for p, (m, mp) in enumerate(pairs(len(mics))):
        out[p] = -(u @ (mics[m] - mics[mp])) * fs / c
    return out


def max_lags(mics, fs, c, n_aux):
    """N_p = floor(Delta t_{p|0} / T) + N_aux with Delta t_{p|0} = d_p / c,
    (33) and (5).  Returns an int array [P]."""
    mics = np.asarray(mics, dtype=np.float64)
    out = []
    for (m, mp) in pairs(len(mics)):
        d = np.sqrt(((mics[m] - mics[mp]) ** 2).sum())
        out.append(int(np.floor(d * fs / c)) + int(n_aux))
    return np.array(out, dtype=np.int64)


def mean_lags(Np):
    """Mean number of samples per pair, N = 1 + (2/P) sum_p N_p, (35)."""
    Np = np.asarray(Np)
    return 1.0 + 2.0 * Np.sum() / len(Np)


# --------------------------------------------------------------------------
# Front end: PHAT-weighted cross-spectra (Sec. II-A, (2))
# --------------------------------------------------------------------------

def phat(Y):
    """Single-sided PHAT-weighted FD GCCs psi_p[l, k] for k = 1..K-1.

    Y: complex STFT frames [L, M, K+1] (bins 0..K of a 2K-point DFT).
    psi_{m,m'} = y_m y_m'^* / |y_m y_m'^*|, (2) with the PHAT weight; 0 where
    the product vanishes.  Returns complex128 [L, P, K-1]."""
    Y = np.asarray(Y).astype(np.complex128)
    L, M, K1 = Y.shape
    K = K1 - 1
    P = M * (M - 1) // 2
    psi = np.zeros((L, P, K - 1), dtype=np.complex128)
    for p, (m, mp) in enumerate(pairs(M)):
        cross = Y[:, m, 1:K] * np.conj(Y[:, mp, 1:K])
        mag = np.abs(cross)
        nz = mag > 0
        psi[:, p, :][nz] = cross[nz] / mag[nz]
    return psi


# --------------------------------------------------------------------------
# Form (a): conv. FD-SRP (Sec. II-D)
# --------------------------------------------------------------------------

def steering(x_p, K):
    """Single-sided SRP matrix block H_p[j, k] = exp(j omega_k Delta t_p(j)),
    k = 1..K-1, (19), with omega_k Delta t = pi k x / K from (1) and (14)."""
    k = np.arange(1, K, dtype=np.float64)
    return np.exp(1j * np.pi * np.outer(x_p, k) / K)


def fd_map(psi, x, K, chunk=4096):
    """conv. FD-SRP map z = 2 Re[H psi], (22), for every frame.

    psi: [L, P, K-1] complex; x: TDOAs in samples [P, J].  Returns [L, J]."""
    psi = np.asarray(psi, dtype=np.complex128)
    L, P, _ = psi.shape
    J = x.shape[1]
    z = np.zeros((L, J), dtype=np.float64)
    for j0 in range(0, J, chunk):
        j1 = min(J, j0 + chunk)
        acc = np.zeros((L, j1 - j0), dtype=np.complex128)
        for p in range(P):
            H = steering(x[p, j0:j1], K)            # [Jc, K-1]
            acc += psi[:, p, :] @ H.T               # sum_k H[j,k] psi[l,k]
        z[:, j0:j1] = 2.0 * acc.real
    return z


def steering_matrix(x, K):
    """The single-sided SRP matrix H = [H_1 ... H_P] of (19)-(21), J x P(K-1),
    columns ordered by pair, then bin k = 1..K-1."""
    return np.concatenate([steering(x[p], K) for p in range(x.shape[0])], axis=1)


def lr_factors(x, K, R):
    """LR-SRP (Sec. II-E): the minimiser of (26) under the rank constraint
    (27), the rank-R truncated SVD of H written as (28).  Returns
    (H_tall = U Sigma [J, R], H_fat = V^H [R, P(K-1)], all singular values)."""
    H = steering_matrix(x, K)
    U, s, Vh = np.linalg.svd(H, full_matrices=False)
    return U[:, :R] * s[:R], Vh[:R].copy(), s


def lr_map(psi, tall, fat):
    """LR-SRP map (29): z = 2 Re[H_tall (H_fat psi)], psi [L, P, K-1]."""
    psi = np.asarray(psi, dtype=np.complex128)
    v = psi.reshape(psi.shape[0], -1)              # stacked (p, k)
    g = v @ fat.T                                  # fat stage [L, R]
    return 2.0 * (g @ tall.T).real                 # tall stage [L, J]


def dsb_power_map(Y, mics, grid, fs, c):
    """Brute-force delay-and-sum output power summed over bins 1..K-1: the
    first line of (8), z(omega, i) = h^H Psi h - tr Psi, with the steering
    vector (7) relative to microphone 1 and the PHAT-weighted Psi of (2).

    Independent of the pair formulation; used to pin fd_map."""
    Y = np.asarray(Y).astype(np.complex128)
    L, M, K1 = Y.shape
    K = K1 - 1
    mics = np.asarray(mics, dtype=np.float64)
    grid = np.asarray(grid, dtype=np.float64)
    dist = np.sqrt(((grid[None, :, :] - mics[:, None, :]) ** 2).sum(-1))
    dt1 = (dist - dist[0:1]) / c                     # Delta t_{m,1}(i)  [M, J]
    J = grid.shape[0]
    z = np.zeros((L, J))
    for k in range(1, K):
        w = np.pi * k * fs / K                        # omega_k = k omega_b / K
        h = np.exp(-1j * w * dt1)                     # [M, J]
        for l in range(L):
            y = Y[l, :, k]
            # Psi = gamma y y^H with the PHAT weight 1/|y_m y_m'^*|
            mag = np.abs(y)
            u = np.zeros(M, dtype=np.complex128)
            u[mag > 0] = y[mag > 0] / mag[mag > 0]
            Psi = np.outer(u, np.conj(u))
            quad = np.einsum("mj,mn,nj->j", np.conj(h), Psi, h)
            z[l] += quad.real - np.trace(Psi).real
    return z


# --------------------------------------------------------------------------
# Sampling (Sec. III-B2, III-B3, Appendix)
# --------------------------------------------------------------------------

def two_sided(psi_p, K):
    """Two-sided GCC bar psi_p over k = -K+1..K in k_mod order (Appendix):
    entry k_mod = mod(k, 2K) holds psi_p(omega_k); the negative bins hold the
    conjugates (real signals), and bins 0 and K are zero."""
    L = psi_p.shape[0]
    bar = np.zeros((L, 2 * K), dtype=np.complex128)
    k = np.arange(1, K)
    bar[:, k] = psi_p
    bar[:, 2 * K - k] = np.conj(psi_p)
    return bar


def gcc_samples_ifft(psi, Np, K):
    """TD GCC samples xi_p(nT), n = -N_p..N_p, by the iFFT of the two-sided
    GCC and lag selection, (46)-(48).  The iFFT is unnormalised (a sum over
    the 2K bins), matching the rows of the iDFT submatrix in (37).

    Returns a list over pairs of real arrays [L, 2 N_p + 1] in natural lag
    order n = -N_p..N_p."""
    out = []
    for p, n_p in enumerate(Np):
        bar = two_sided(psi[:, p, :], K)
        full = np.fft.ifft(bar, axis=1) * (2 * K)     # unnormalised iFFT
        n = np.arange(-n_p, n_p + 1)
        out.append(full[:, np.mod(n, 2 * K)].real)
    return out


def gcc_samples_direct(psi, Np, K):
    """The same samples by the matrix-vector product xi_p = 2 Re[S_p psi_p],
    (40), with [S_p]_{n,k} = exp(j pi k n / K), (37)."""
    out = []
    k = np.arange(1, K, dtype=np.float64)
    for p, n_p in enumerate(Np):
        n = np.arange(-n_p, n_p + 1, dtype=np.float64)
        S = np.exp(1j * np.pi * np.outer(n, k) / K)   # [2N_p+1, K-1]
        out.append(2.0 * (psi[:, p, :] @ S.T).real)
    return out


def stack_samples(xi_list):
    """Stacked xi in R^{PN} per frame, (38)."""
    return np.concatenate(xi_list, axis=1)


# --------------------------------------------------------------------------
# Interpolation: SI, TD, SLRI, SSPI (Sec. II-E, III-B, IV-A)
# --------------------------------------------------------------------------

def interp_matrix(x_p, n_p):
    """Interpolation matrix Lambda_p[j, n] = sinc(Delta t_p(j)/T - n) over
    n = -N_p..N_p (natural order), (42)."""
    n = np.arange(-n_p, n_p + 1, dtype=np.float64)
    return np.sinc(np.subtract.outer(np.asarray(x_p, dtype=np.float64), n))


def si_map(xi_list, x, Np):
    """SI-SRP map z_si = sum_p Lambda_p xi_p, (44)."""
    L = xi_list[0].shape[0]
    z = np.zeros((L, x.shape[1]))
    for p, n_p in enumerate(Np):
        z += xi_list[p] @ interp_matrix(x[p], n_p).T
    return z


def td_map(xi_list, x, Np):
    """conv. TD-SRP map, (23): the GCC read at the TDOA rounded to the nearest
    sample.  Rounding half away from zero; the lag is kept in the sampled
    range [-N_p, N_p] (with N_aux = 0 an endfire TDOA can round to N_p + 1,
    which the sampling of (46)-(48) does not hold)."""
    L = xi_list[0].shape[0]
    z = np.zeros((L, x.shape[1]))
    for p, n_p in enumerate(Np):
        n = np.sign(x[p]) * np.floor(np.abs(x[p]) + 0.5)
        n = np.clip(n, -n_p, n_p)
        idx = (n + n_p).astype(np.int64)
        z += xi_list[p][:, idx]
    return z


def slri_factors(x, Np, R):
    """Per-pair low-rank interpolation: rank-R_p truncated SVD of each
    Lambda_p, R_p = min(R, 2 N_p + 1), the minimiser of (54) restricted to
    one pair.  Returns a list of (U_p [J, R_p] = U Sigma, V_p [2N_p+1, R_p],
    singular values)."""
    out = []
    for p, n_p in enumerate(Np):
        lam = interp_matrix(x[p], n_p)
        U, s, Vt = np.linalg.svd(lam, full_matrices=False)
        r = min(int(R), 2 * int(n_p) + 1)
        out.append((U[:, :r] * s[:r], Vt[:r].T.copy(), s))
    return out


def slri_factors_gram(x, Np, R, cols, chunk=16384):
    """The same per-pair rank-R_p truncation computed through the Gram
    matrix: the right singular vectors of Lambda_p are the eigenvectors of
    Lambda_p^T Lambda_p and its eigenvalues the squared singular values (the
    SVD of (54) written as an eigenproblem), so V_p needs only the
    (2N_p+1)^2 Gram matrix, accumulated over candidates in chunks.  U_p =
    Lambda_p V_p is returned for the candidates `cols` only.  For problems
    whose Lambda_p is too tall to decompose directly."""
    out = []
    J = x.shape[1]
    for p, n_p in enumerate(Np):
        n = 2 * int(n_p) + 1
        G = np.zeros((n, n))
        for j0 in range(0, J, chunk):
            lam = interp_matrix(x[p, j0:j0 + chunk], n_p)
            G += lam.T @ lam
        w, v = np.linalg.eigh(G)
        order = np.argsort(w)[::-1]
        w, v = w[order], v[:, order]
        r = min(int(R), n)
        V = v[:, :r]
        U = interp_matrix(x[p, cols], n_p) @ V
        out.append((U, V, np.sqrt(np.maximum(w, 0.0))))
    return out


def slri_map(xi_list, factors):
    """SLRI-SRP map, per-pair form of (57): z = sum_p U_p (V_p^T xi_p)."""
    L = xi_list[0].shape[0]
    J = factors[0][0].shape[0]
    z = np.zeros((L, J))
    for xi_p, (U_p, V_p, _) in zip(xi_list, factors):
        g = xi_p @ V_p                                # fat stage  [L, R_p]
        z += g @ U_p.T                                # tall stage [L, J]
    return z


def slri_global_factors(x, Np, R):
    """Global low-rank interpolation of (54), (56): rank-R truncated SVD of the
    stacked Lambda (43) of size J x PN.  Returns (Lambda_tall, Lambda_fat)."""
    lam = np.concatenate([interp_matrix(x[p], n_p) for p, n_p in enumerate(Np)], axis=1)
    U, s, Vt = np.linalg.svd(lam, full_matrices=False)
    return U[:, :R] * s[:R], Vt[:R].copy()


def slri_global_map(xi_list, tall, fat):
    """SLRI-SRP map of (57): z = Lambda_tall (Lambda_fat xi)."""
    xi = stack_samples(xi_list)
    return (xi @ fat.T) @ tall.T


def sspi_select(x_p, n_p, Q):
    """Per-(location, pair) sparse interpolation: keep the Q_p = min(Q, 2N_p+1)
    entries of each row of Lambda_p with the largest magnitude, no refit, the
    minimiser of (55) with Q_p nonzeros per row.  Ties go to the smaller
    |x - n|, then to the smaller n (a stable lexicographic sort).

    Returns (lags [J, Q_p] int64, weights [J, Q_p] float64), lags in
    ascending order per row."""
    lam = interp_matrix(x_p, n_p)                     # [J, 2N_p+1]
    n = np.arange(-n_p, n_p + 1)
    q = min(int(Q), 2 * int(n_p) + 1)
    dist = np.abs(np.subtract.outer(np.asarray(x_p, dtype=np.float64), n.astype(np.float64)))
    nn = np.broadcast_to(n, lam.shape)
    # Magnitudes equal to 13 decimals count as ties: sinc at a nonzero integer
    # is exactly zero in the definition but ~1e-17 in floating point.
    mag = np.round(np.abs(lam), 13)
    # np.lexsort sorts by the last key first: -|Lambda|, then |x - n|, then n;
    # it sorts every row independently along the last axis.
    order = np.lexsort((nn, dist, -mag), axis=-1)[:, :q]
    order = np.sort(order, axis=1)
    lags = n[order]
    wts = np.take_along_axis(lam, order, axis=1)
    return lags, wts


def sspi_map(xi_list, selections, Np):
    """SSPI-SRP map of (58) in the per-(location, pair) form:
    z[l, j] = sum_p sum_{n in sel(j,p)} Lambda_p[j, n] xi_p[l, n]."""
    L = xi_list[0].shape[0]
    J = selections[0][0].shape[0]
    z = np.zeros((L, J))
    for xi_p, (lags, wts), n_p in zip(xi_list, selections, Np):
        for q in range(lags.shape[1]):
            z += xi_p[:, lags[:, q] + n_p] * wts[:, q][None, :]
    return z


def sspi_global_select(x, Np, Q_total):
    """Global sparse interpolation of (55): keep the Q_Lambda largest-magnitude
    entries of the stacked Lambda (43).  Returns the sparse matrix as a dense
    J x PN array with the discarded entries set to zero."""
    lam = np.concatenate([interp_matrix(x[p], n_p) for p, n_p in enumerate(Np)], axis=1)
    flat = np.abs(lam).ravel()
    keep = np.argsort(-flat, kind="stable")[: int(Q_total)]
    sp = np.zeros_like(lam).ravel()
    sp[keep] = lam.ravel()[keep]
    return sp.reshape(lam.shape)


def sspi_global_map(xi_list, lam_sp):
    """SSPI-SRP map of (58): z = Lambda_sp xi."""
    return stack_samples(xi_list) @ lam_sp.T


def periodic_interp_map(xi_full, x, K):
    """Map from all 2K samples of each GCC through the exact periodic
    interpolator of a signal whose DC and Nyquist bins are zero:
    xi(t) = sum_n xi[n] D(t - n), D(t) = sin((K - 1/2) pi t / K) /
    (2K sin(pi t / (2K))).  With DC and Nyquist zero this reproduces the
    conv. FD-SRP map (22) exactly; used only as a pin.

    xi_full: [L, P, 2K] unnormalised iFFT outputs."""
    L, P, N = xi_full.shape
    z = np.zeros((L, x.shape[1]))
    n = np.arange(N, dtype=np.float64)
    for p in range(P):
        t = np.subtract.outer(x[p], n)               # [J, 2K]
        num = np.sin((K - 0.5) * np.pi * t / K)
        den = 2 * K * np.sin(np.pi * t / (2 * K))
        D = np.empty_like(t)
        small = np.abs(den) < 1e-300
        D[~small] = num[~small] / den[~small]
        D[small] = (2 * K - 1) / (2 * K)
        z += xi_full[:, p, :] @ D.T
    return z


# --------------------------------------------------------------------------
# Peak picking and error measures (Sec. II-B, Sec. V-A)
# --------------------------------------------------------------------------

def argmax_map(z):
    """Candidate index maximising each map, (11); ties to the smallest index."""
    return np.argmax(np.asarray(z), axis=-1)


def rel_error(z, z_ref):
    """Per-map relative error ||z - z_ref|| / ||z_ref||."""
    z = np.asarray(z, dtype=np.float64)
    z_ref = np.asarray(z_ref, dtype=np.float64)
    return np.linalg.norm(z - z_ref, axis=-1) / np.linalg.norm(z_ref, axis=-1)


def eps_z_db(z, z_ref):
    """Map error epsilon_z in dB, (65)."""
    return 20.0 * np.log10(rel_error(z, z_ref))


def eps_h_db(H_type, H):
    """Matrix error epsilon_H in dB, (64)."""
    return 10.0 * np.log10(np.sum(np.abs(H_type - H) ** 2) / np.sum(np.abs(H) ** 2))


# --------------------------------------------------------------------------
# Complexity model (Sec. II-F, III-A2, III-B3, IV-B)
# --------------------------------------------------------------------------

def complexity(J, P, K, N=None, R_lambda=None, Q_lambda=None, R_H=None,
               sampling="ifft"):
    """Real MAC counts per map.  C of (24); C_td of (25) with the pair count
    P multiplying the iFFT term (the term as printed lacks it; Fig. 12's
    values need it); C_lr of (30); C_samp of (49); C_si of (50); C_slri and
    C_sspi of (61), (62)."""
    C = 2 * J * P * (K - 1)
    log2 = np.log2(2 * K)
    if sampling == "ifft":
        c_samp = 8 * P * K * log2
    else:
        c_samp = 2 * P * N * (K - 1)
    out = {"C": C, "C_samp": c_samp, "C_td": J * P + 8 * P * K * log2}
    if N is not None:
        out["C_si"] = J * P * N + c_samp
    if R_lambda is not None and N is not None:
        out["C_slri"] = J * R_lambda + R_lambda * P * N + c_samp
    if Q_lambda is not None:
        out["C_sspi"] = Q_lambda + c_samp
    if R_H is not None:
        out["C_lr"] = 2 * J * R_H + 4 * R_H * P * (K - 1)
    return out
