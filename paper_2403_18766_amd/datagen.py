"""Seeded synthetic workloads (the inputs every test, the benchmark and the
oracle share).  Nothing here computes any part of the clustering method.

The paper evaluates on 23 public data sets (Section 5) that are not shipped
with this code; these generators stand in for them with the shapes the
method meets there: 2 to several hundred attributes, 10^4 to 10^7 points,
well-separated and overlapping clusters, background noise, and unit-norm
embedding-like data.

All generators draw in FP64 from ``numpy.random.default_rng(seed)``, shuffle
the rows and return C-contiguous FP32 arrays (the storage precision of X).
"""

import hashlib

import numpy as np


def _shuffle_f32(rng, X):
    perm = rng.permutation(X.shape[0])
    return np.ascontiguousarray(X[perm], dtype=np.float32)


def isotropic_blobs(m, n, n_centres, seed=0, box=10.0, sigma=1.0, equal=True):
    """Isotropic Gaussian blobs: centres ~ U[-box, box]^n, x = mu + N(0, sigma^2 I).

    equal=True gives every blob m // n_centres points (the remainder to the
    first ones); otherwise weights ~ Dirichlet(1)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-box, box, size=(n_centres, n))
    if equal:
        counts = np.full(n_centres, m // n_centres)
        counts[: m - counts.sum()] += 1
    else:
        counts = rng.multinomial(m, rng.dirichlet(np.ones(n_centres)))
    parts = [mu[j] + sigma * rng.standard_normal((counts[j], n)) for j in range(n_centres)]
    return _shuffle_f32(rng, np.concatenate(parts, axis=0))


def anisotropic_mixture(m, n, n_centres, seed=0, box=20.0, eig=(0.5, 4.0)):
    """Gaussian mixture with random covariances Q diag(lambda) Q^T, lambda ~ U[eig]^n,
    Q Haar-distributed; centres ~ U[-box, box]^n; weights ~ Dirichlet(1)."""
    from scipy.stats import ortho_group
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-box, box, size=(n_centres, n))
    w = rng.dirichlet(np.ones(n_centres))
    counts = rng.multinomial(m, w)
    X = np.empty((m, n), dtype=np.float64)
    row = 0
    for j in range(n_centres):
        lam = rng.uniform(eig[0], eig[1], size=n)
        Q = ortho_group.rvs(n, random_state=rng) if n > 1 else np.ones((1, 1))
        z = rng.standard_normal((counts[j], n))
        X[row: row + counts[j]] = mu[j] + (z * np.sqrt(lam)) @ Q.T
        row += counts[j]
    return _shuffle_f32(rng, X)


def noisy_mixture(m, n, n_centres, seed=0, box=20.0, sigma=(0.5, 3.0), noise=0.05):
    """Isotropic Gaussians with sigma_j ~ U[sigma], centres ~ U[-box, box]^n,
    weights ~ Dirichlet(1), plus a fraction `noise` of points uniform in the
    per-dimension bounding box of the Gaussian points."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-box, box, size=(n_centres, n))
    sig = rng.uniform(sigma[0], sigma[1], size=n_centres)
    n_noise = int(round(noise * m))
    counts = rng.multinomial(m - n_noise, rng.dirichlet(np.ones(n_centres)))
    X = np.empty((m, n), dtype=np.float64)
    row = 0
    for j in range(n_centres):
        X[row: row + counts[j]] = mu[j] + sig[j] * rng.standard_normal((counts[j], n))
        row += counts[j]
    g = X[:row]
    lo, hi = g.min(axis=0), g.max(axis=0)
    X[row:] = rng.uniform(lo, hi, size=(n_noise, n))
    return _shuffle_f32(rng, X)


def vmf_mixture(per_cluster, n, n_centres, seed=0, kappa=(50.0, 200.0)):
    """Unit-norm points from a mixture of von Mises-Fisher components on S^(n-1):
    mean directions are normalised N(0, I) vectors, kappa_j ~ U[kappa]; each
    point is re-normalised in FP64 before the FP32 store."""
    from scipy.stats import vonmises_fisher
    rng = np.random.default_rng(seed)
    X = np.empty((per_cluster * n_centres, n), dtype=np.float32)
    for j in range(n_centres):
        mu = rng.standard_normal(n)
        mu /= np.linalg.norm(mu)
        kap = rng.uniform(kappa[0], kappa[1])
        pts = vonmises_fisher(mu, kap).rvs(per_cluster, random_state=rng)
        pts /= np.linalg.norm(pts, axis=1, keepdims=True)
        X[j * per_cluster: (j + 1) * per_cluster] = pts
    perm = rng.permutation(X.shape[0])
    return np.ascontiguousarray(X[perm])


def _vmf_cosines(rng, kappa, p, size):
    """Cosines w = x.mu of `size` vMF(mu, kappa) points on S^(p-1): Wood's (1994)
    rejection sampler, vectorised."""
    b = (p - 1) / (2.0 * kappa + np.sqrt(4.0 * kappa * kappa + (p - 1) ** 2))
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + (p - 1) * np.log(1.0 - x0 * x0)
    out = np.empty(size)
    filled = 0
    while filled < size:
        nd = int((size - filled) * 1.25) + 16
        z = rng.beta((p - 1) / 2.0, (p - 1) / 2.0, nd)
        u = rng.uniform(size=nd)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        ok = kappa * w + (p - 1) * np.log(1.0 - x0 * w) - c >= np.log(u)
        w = w[ok][: size - filled]
        out[filled: filled + w.size] = w
        filled += w.size
    return out


def vmf_mixture_device(per_cluster, n, n_centres, device, seed=0, kappa=(50.0, 200.0)):
    """The vmf_mixture recipe drawn on a torch device (for sizes the host
    sampler is too slow for): mean directions and kappa from
    default_rng(seed), the cosine to the mean direction by Wood's sampler, the
    tangent direction from a seeded torch generator on the device; points are
    re-normalised in FP64 and stored FP32, rows shuffled.  Returns an
    (per_cluster * n_centres) x n float32 tensor on the device."""
    import torch
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    m = per_cluster * n_centres
    X = torch.empty((m, n), dtype=torch.float32, device=device)
    for j in range(n_centres):
        mu = rng.standard_normal(n)
        mu /= np.linalg.norm(mu)
        kap = rng.uniform(kappa[0], kappa[1])
        w = torch.from_numpy(_vmf_cosines(rng, kap, n, per_cluster)).to(device)[:, None]
        mu_t = torch.from_numpy(mu).to(device)
        v = torch.randn((per_cluster, n), generator=gen, device=device, dtype=torch.float64)
        v -= (v @ mu_t)[:, None] * mu_t[None, :]
        v /= torch.linalg.vector_norm(v, dim=1, keepdim=True)
        x = w * mu_t[None, :] + torch.sqrt(torch.clamp(1.0 - w * w, min=0.0)) * v
        x /= torch.linalg.vector_norm(x, dim=1, keepdim=True)
        X[j * per_cluster: (j + 1) * per_cluster] = x.to(torch.float32)
    perm = torch.from_numpy(rng.permutation(m)).to(device)
    return X.index_select(0, perm)


def vmf_mixture_host(per_cluster, n, n_centres, seed=0, kappa=(50.0, 200.0), threads=None):
    """The vmf_mixture_device recipe on the host, reproducible bit for bit on
    any machine with this NumPy: mean directions, kappa and the row order from
    default_rng(seed); cluster j's cosines (Wood's sampler) and tangent
    directions from its own stream default_rng([seed, 1 + j]), so clusters
    are drawn in parallel threads and the result does not depend on their
    number.  Points are normalised in FP64 and stored FP32."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(seed)
    mus, kaps = [], []
    for _ in range(n_centres):
        mu = rng.standard_normal(n)
        mus.append(mu / np.linalg.norm(mu))
        kaps.append(rng.uniform(kappa[0], kappa[1]))
    m = per_cluster * n_centres
    X = np.empty((m, n), dtype=np.float32)

    def one(j):
        r = np.random.default_rng([seed, 1 + j])
        mu = mus[j]
        w = _vmf_cosines(r, kaps[j], n, per_cluster)[:, None]
        v = r.standard_normal((per_cluster, n))
        v -= (v @ mu)[:, None] * mu[None, :]
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        x = w * mu[None, :] + np.sqrt(np.clip(1.0 - w * w, 0.0, None)) * v
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        X[j * per_cluster: (j + 1) * per_cluster] = x

    if threads is None:
        threads = min(16, len(os.sched_getaffinity(0)))
    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(one, range(n_centres)))
    perm = rng.permutation(m)
    return np.ascontiguousarray(X[perm])


# The five workloads (sizes of the configurations this code is measured on).
WORKLOADS = {
    "blobs2d": dict(desc="20,000 points in 2-D from 5 isotropic Gaussians (centres U[-10,10]^2, "
                         "sigma 1, equal weights); k=5",
                    m=20_000, n=2, k=5),
    "aniso28": dict(desc="1,000,000 points in 28-D from 25 anisotropic Gaussians (eigenvalues "
                         "U[0.5,4], centres U[-20,20]^28, Dirichlet(1) weights); k=25",
                    m=1_000_000, n=28, k=25),
    "noisy28": dict(desc="10,000,000 points in 28-D from 50 Gaussians (sigma U[0.5,3]) plus 5% "
                         "uniform background noise; k=50",
                    m=10_000_000, n=28, k=50),
    "vmf768": dict(desc="2,000,000 unit vectors in 768-D from 100 von Mises-Fisher clusters "
                        "(kappa U[50,200]); k=100",
                   m=2_000_000, n=768, k=100),
}


def make(name, seed=0, m=None):
    """Build one named workload (optionally with fewer points, same recipe)."""
    w = WORKLOADS[name]
    mm = w["m"] if m is None else int(m)
    if name == "blobs2d":
        return isotropic_blobs(mm, 2, 5, seed=seed, box=10.0, sigma=1.0, equal=True)
    if name == "aniso28":
        return anisotropic_mixture(mm, 28, 25, seed=seed)
    if name == "noisy28":
        return noisy_mixture(mm, 28, 50, seed=seed)
    if name == "vmf768":
        if m is None:   # the measured workload: reproducible host generator
            return vmf_mixture_host(mm // 100, 768, 100, seed=seed)
        return vmf_mixture(max(1, mm // 100), 768, 100, seed=seed)
    raise KeyError(name)


def serving_dataset(n, m=4_000_000, seed=0):
    """Resident data set of the serving workload: the noisy-mixture recipe in dimension n."""
    return noisy_mixture(m, n, 50, seed=seed)


def sha256(X):
    return hashlib.sha256(np.ascontiguousarray(X).tobytes()).hexdigest()


def sha256_chunked(X, chunk=1 << 26):
    """sha256 of the concatenated sha256 digests of X's bytes in chunks of
    `chunk` bytes (chunks hashed in parallel threads; for multi-GB inputs)."""
    from concurrent.futures import ThreadPoolExecutor
    buf = memoryview(np.ascontiguousarray(X)).cast("B")
    parts = [buf[o: o + chunk] for o in range(0, len(buf), chunk)]
    with ThreadPoolExecutor(8) as ex:
        digests = list(ex.map(lambda b: hashlib.sha256(b).digest(), parts))
    return hashlib.sha256(b"".join(digests)).hexdigest()
