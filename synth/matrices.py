"""Matrix generators (NumPy, float64).

haar(m, n, rng): m x n matrix with orthonormal columns, Haar distributed
    (QR of a Gaussian with the signs of diag(R) moved into Q; Mezzadri 2007).
spectrum_matrix(m, n, sigma, seed): U diag(sigma) V^T with Haar U, V.
lowrank_noise(...): spectrum_matrix + i.i.d. Gaussian noise.
gauss_kernel(n, d, seed): K_ij = exp(-|x_i - x_j|^2 / (2 h^2)), x_i ~ N(0, I_d),
    h = median pairwise distance of a subsample.
"""
import numpy as np


def haar(m, n, rng):
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def spectrum_matrix(m, n, sigma, seed):
    rng = np.random.default_rng(seed)
    r = len(sigma)
    U = haar(m, r, rng)
    V = haar(n, r, rng)
    return (U * np.asarray(sigma, dtype=np.float64)[None, :]) @ V.T


def lowrank_noise(m, n, sigma, noise_std, seed):
    A = spectrum_matrix(m, n, sigma, seed)
    if noise_std:
        rng = np.random.default_rng(seed + 7919)
        A = A + noise_std * rng.standard_normal((m, n))
    return A


def psd_from_spectrum(n, lam, seed):
    rng = np.random.default_rng(seed)
    U = haar(n, len(lam), rng)
    return (U * np.asarray(lam, dtype=np.float64)[None, :]) @ U.T


def gauss_kernel(n, d, seed, sub=4096):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Xs = X[: min(sub, n)]
    sq = np.sum(Xs * Xs, axis=1)
    D2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * Xs @ Xs.T, 0.0)
    iu = np.triu_indices(Xs.shape[0], 1)
    h = float(np.median(np.sqrt(D2[iu])))
    sqa = np.sum(X * X, axis=1)
    D2a = np.maximum(sqa[:, None] + sqa[None, :] - 2.0 * X @ X.T, 0.0)
    K = np.exp(-D2a / (2.0 * h * h))
    np.fill_diagonal(K, 1.0)
    return K


# Workload presets.  "full" sizes are what the benchmark runs; the parity tests
# use the "small" versions (same spectra laws, sizes the oracle finishes in
# seconds).
WORKLOADS = {
    # dense FP64 2000 x 1000, sigma_i = 1/i, noise N(0, 1e-6) per entry (variance)
    "cpu2000": dict(m=2000, n=1000, law="inv", p=1.0, noise_var=1e-6, k=50, l=100, s=8, q=2, seed=101),
    # 65536 x 16384 FP32, sigma_i = i^-1.5, noise of spectral size 1e-4 sigma_1
    "poly65k": dict(m=65536, n=16384, law="poly", p=1.5, noise_spec=1e-4, k=1000, l=2000, s=8, q=2, seed=102),
    # 65536 x 32768, sigma_i = max(0.995^i, 1e-3 sigma_1)
    "exp65k": dict(m=65536, n=32768, law="expfloor", base=0.995, floor=1e-3, k=2000, l=4000, s=8, q=3, seed=103),
    # the paper's synthetic "polydecay" (Section 4): 30000 x 15000, sigma_i = 30000 / i,
    # random orthogonal factors, no noise; k = 40, l in {800, 1200, 1600}, CountSketch
    "polydecay": dict(m=30000, n=15000, law="inv", scale=30000.0, k=40, l=800, s=1, q=2, seed=106),
}


def sigma_law(law, r, p=1.0, base=0.995, floor=1e-3):
    i = np.arange(1, r + 1, dtype=np.float64)
    if law == "inv":
        return 1.0 / i
    if law == "poly":
        return i ** (-p)
    if law == "expfloor":
        s = base ** i
        return np.maximum(s, floor * s[0])
    raise ValueError(law)


def workload(name, m=None, n=None, seed=None):
    """NumPy instance of a preset at (possibly reduced) size.  Returns (A, spec)."""
    w = dict(WORKLOADS[name])
    m = w["m"] if m is None else m
    n = w["n"] if n is None else n
    seed = w["seed"] if seed is None else seed
    r = min(m, n)
    sig = w.get("scale", 1.0) * sigma_law(w["law"], r, w.get("p", 1.0), w.get("base", 0.995), w.get("floor", 1e-3))
    std = 0.0
    if "noise_var" in w:
        std = float(np.sqrt(w["noise_var"]))
    elif "noise_spec" in w:
        std = w["noise_spec"] * sig[0] / (np.sqrt(m) + np.sqrt(n))
    A = lowrank_noise(m, n, sig, std, seed)
    return A, dict(w, m=m, n=n, seed=seed, sigma=sig, noise_std=std)
