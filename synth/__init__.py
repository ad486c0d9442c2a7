"""Seeded synthetic inputs for the LDDMM hot path (shared by the tests, the
benchmark, the smoke check and the oracle runs).

This module holds input generators only -- none of the registration method's
arithmetic (no transport, no spectral operator of the method, no
interpolation).  Every field is returned as float64; callers cast to float32
for the GPU and hand the same float32 values (up-cast) to the oracle.

Stand-ins: the paper's experiments use NIREP T1 brain MR volumes (256x300x256
resampled to 256^3, intensities in [0,1]) and CLARITY volumes; neither is
available here, so smooth blob images with the same size and intensity range
stand in for them, and band-limited random velocities with a prescribed
maximum displacement stand in for registration velocities.
"""
import numpy as np


def _half_space_modes(K):
    """Integer wave vectors k with 0 < |k| <= K in the half space
    (k1 > 0) or (k1 = 0, k2 > 0) or (k1 = k2 = 0, k3 > 0)."""
    r = np.arange(-K, K + 1)
    k = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    kk = (k ** 2).sum(1)
    half = (k[:, 0] > 0) | ((k[:, 0] == 0) & (k[:, 1] > 0)) | (
        (k[:, 0] == 0) & (k[:, 1] == 0) & (k[:, 2] > 0))
    return k[(kk > 0) & (kk <= K * K) & half]


def _evaluate_modes(shape, K, coef):
    """Re sum_k coef[..., k] exp(i k.x) on the grid, separably along each
    axis.  coef: complex array [ncomp][2K+1][2K+1][2K+1] indexed by k+K."""
    n1, n2, n3 = shape
    x = [np.arange(n) * (2 * np.pi / n) for n in shape]
    r = np.arange(-K, K + 1)
    E = [np.exp(1j * np.outer(xi, r)) for xi in x]  # [n][2K+1]
    out = []
    for c in coef:
        s3 = np.einsum("abk,zk->abz", c, E[2])          # k1,k2,x3
        s2 = np.einsum("abz,yb->ayz", s3, E[1])  # k1,x2,x3
        s1 = (E[0] @ s2.reshape(2 * K + 1, -1)).reshape(n1, n2, n3)
        out.append(s1.real)
    return np.stack(out)


def bandlimited_vector(shape, K, seed, max_disp=None, divfree=False, ncomp=3):
    """Band-limited random field v_c = sum_{0<|k|<=K} a cos(k.x) + b sin(k.x),
    a, b ~ N(0,1)/(1+|k|^2).  divfree: v = curl(psi) with psi drawn the same
    way.  max_disp: scale so that max_x |v(x)| = max_disp * h (h = 2pi/min n),
    i.e. a displacement of about max_disp voxels over unit time."""
    rng = np.random.default_rng(seed)
    modes = _half_space_modes(K)
    amp = 1.0 / (1.0 + (modes ** 2).sum(1))
    nc = 3 if divfree else ncomp
    a = rng.standard_normal((nc, len(modes))) * amp
    b = rng.standard_normal((nc, len(modes))) * amp
    hat = a - 1j * b  # Re(hat e^{ik.x}) = a cos + b sin
    if divfree:
        hat = _curl_hat(modes, hat)
    coef = np.zeros((hat.shape[0], 2 * K + 1, 2 * K + 1, 2 * K + 1), complex)
    idx = tuple((modes + K).T)
    for c in range(hat.shape[0]):
        coef[c][idx] = hat[c]
    v = _evaluate_modes(shape, K, coef)
    if max_disp is not None:
        vmax = np.sqrt((v ** 2).sum(0)).max() if v.shape[0] == 3 else np.abs(v).max()
        v *= max_disp * (2 * np.pi / min(shape)) / vmax
    return v


def _curl_hat(modes, hat):
    """Fourier coefficients of curl(psi): i k x psi_hat, per mode."""
    k = modes.astype(float)
    p = hat.T  # [nmodes][3]
    c = np.cross(k, p)
    return (1j * c).T


def bandlimited_scalar(shape, K, seed):
    """One band-limited random scalar field, normalised to max |f| = 1."""
    f = bandlimited_vector(shape, K, seed, ncomp=1)[0]
    return f / np.abs(f).max()


def unit_rms(v):
    return v / np.sqrt(np.mean(v ** 2))


def _periodic_gauss(n, centre, sigma):
    """1D periodic Gaussian profile on n grid points (voxel units), summed
    over the nearest periodic images."""
    i = np.arange(n, dtype=float)
    g = np.zeros(n)
    for s in (-1, 0, 1):
        g += np.exp(-0.5 * ((i - centre + s * n) / sigma) ** 2)
    return g


def blob_image(shape, nblobs, seed, sigma=(3.0, 12.0)):
    """Smooth 'brain-like' image: sum of separable periodic Gaussian blobs,
    centres uniform on the grid, sigma ~ U[3,12] voxels, amplitude ~ U[0,1],
    min-max normalised to [0,1]."""
    rng = np.random.default_rng(seed)
    img = np.zeros(shape)
    for _ in range(nblobs):
        c = rng.uniform(0, 1, 3) * np.array(shape)
        s = rng.uniform(sigma[0], sigma[1])
        A = rng.uniform(0, 1)
        prof = [_periodic_gauss(n, c[d], s) for d, n in enumerate(shape)]
        sup = [np.nonzero(p > 1e-14)[0] for p in prof]
        blk = A * prof[0][sup[0]][:, None, None] * prof[1][sup[1]][None, :, None] \
            * prof[2][sup[2]][None, None, :]
        img[np.ix_(*sup)] += blk
    img -= img.min()
    return img / img.max()


def sin2_template(shape, K=4, seed=1000, noise=0.1):
    """m0 = prod_i sin^2(x_i/2) + noise * f, f band-limited (|k| <= K),
    max |f| = 1 (the 32^3 parity problem)."""
    x = np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")
    m0 = np.sin(x[0] / 2) ** 2 * np.sin(x[1] / 2) ** 2 * np.sin(x[2] / 2) ** 2
    return m0 + noise * bandlimited_scalar(shape, K, seed)


def syn_problem(shape):
    """The paper's SYN test problem (Section 4): m0 = sum_i sin^2(x_i)/3 and
    the divergence-free velocity v_l = sin(x_i) cos(x_k) sin(x_k),
    (i,k) = (3,2), (1,3), (2,1) for l = 1,2,3 (1-based axes)."""
    x = np.meshgrid(*[np.arange(n) * (2 * np.pi / n) for n in shape], indexing="ij")
    m0 = sum(np.sin(xi) ** 2 for xi in x) / 3.0
    pairs = [(2, 1), (0, 2), (1, 0)]
    v = np.stack([np.sin(x[i]) * np.cos(x[k]) * np.sin(x[k]) for i, k in pairs])
    return m0, v


def f32(a):
    """float32 copy (what the GPU gets) ..."""
    return np.ascontiguousarray(a, dtype=np.float32)


def f64(a):
    """... and the same values up-cast for the oracle."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
