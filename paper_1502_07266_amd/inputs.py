"""Seeded synthetic inputs shared by the HIP path's tests, the bench and the oracle's tests.

This module only *makes inputs* (velocity models, source vectors, receiver data layout and
the sweep parameters of each named workload).  It holds none of the method's arithmetic and
imports neither the HIP binding nor the oracle.

Arrays are indexed [k, j, i] = (x3, x2, x1) with x1 fastest, matching the column-major
unknown ordering of Sec. 3 of the paper.  Node (i, j, k) sits at (i h, j h, k h), h = 1/(n+1).

Seeds: medium 0, sources 1, medium perturbation 2, finite-difference cells 3.

The paper's own velocity models (a Gaussian lens, a Gaussian waveguide, a random field) and
its Gaussian sources were only shown as figures; the models below are synthetic stand-ins
with the same grid sizes, the same 8 points per wavelength and the same omega/2pi.
"""
import math

import numpy as np

SEED_MEDIUM, SEED_SOURCES, SEED_PERTURB, SEED_FDCELLS = 0, 1, 2, 3


def grid_h(n):
    return 1.0 / (n + 1)


def _coords(n):
    h = grid_h(n)
    x = np.arange(1, n + 1) * h
    return np.meshgrid(x, x, x, indexing="ij")[::-1]   # returns (X1, X2, X3) each [k, j, i]


def medium_constant(n, c0=1.0):
    return np.full((n, n, n), float(c0))


def medium_lens(n, amplitude=-0.4):
    """Gaussian lens c = 1 + amplitude exp(-|x - 0.5|^2 / 0.02) at the nodes (low-velocity
    for amplitude < 0)."""
    X1, X2, X3 = _coords(n)
    r2 = (X1 - 0.5) ** 2 + (X2 - 0.5) ** 2 + (X3 - 0.5) ** 2
    return 1.0 + amplitude * np.exp(-r2 / 0.02)


def medium_waveguide(n, amplitude=-0.4):
    """Vertical Gaussian waveguide, constant along x3:
    c = 1 + amplitude exp(-((x1 - 0.5)^2 + (x2 - 0.5)^2) / 0.02)."""
    X1, X2, _ = _coords(n)
    return 1.0 + amplitude * np.exp(-((X1 - 0.5) ** 2 + (X2 - 0.5) ** 2) / 0.02)


def force_gaussian(n, center, sigma):
    """Smooth point-like source exp(-|x - center|^2 / (2 sigma^2)) at the nodes (complex128)."""
    X1, X2, X3 = _coords(n)
    r2 = (X1 - center[0]) ** 2 + (X2 - center[1]) ** 2 + (X3 - center[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma ** 2)).astype(np.complex128)


def force_wave_packet(n, center, direction, omega, sigma):
    """Gaussian wave packet exp(-|x - center|^2 / (2 sigma^2)) exp(i omega direction . x):
    a plane wave of wavelength 2 pi / omega (that of c = 1) travelling along `direction`."""
    X1, X2, X3 = _coords(n)
    r2 = (X1 - center[0]) ** 2 + (X2 - center[1]) ** 2 + (X3 - center[2]) ** 2
    phase = omega * (direction[0] * X1 + direction[1] * X2 + direction[2] * X3)
    return np.exp(-r2 / (2.0 * sigma ** 2)) * np.exp(1j * phase)


def medium_grf(n, corr_len, lo, hi, seed=SEED_MEDIUM):
    """Gaussian random field with covariance ~ exp(-r^2 / (2 corr_len^2)), mapped onto [lo, hi].

    iid N(0,1) on the nodes, periodic FFT convolution with a Gaussian kernel of standard
    deviation corr_len/sqrt(2), standardised, then an affine min-max map onto [lo, hi].
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    h = grid_h(n)
    sd = corr_len / math.sqrt(2.0)
    k = np.fft.fftfreq(n, d=h) * 2.0 * np.pi
    K3, K2, K1 = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-0.5 * sd ** 2 * (K1 ** 2 + K2 ** 2 + K3 ** 2))
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g = (g - g.mean()) / g.std()
    return lo + (hi - lo) * (g - g.min()) / (g.max() - g.min())


def medium_two_layer(n, c_low=1.0, c_high=1.5, pert=0.05, seed=SEED_PERTURB):
    """c0 = c_low for x3 < 0.5 and c_high above, times (1 + pert * U(-1, 1)) iid per node.
    Returns (c, c0)."""
    X1, X2, X3 = _coords(n)
    c0 = np.where(X3 < 0.5, c_low, c_high).astype(np.float64)
    rng = np.random.default_rng(seed)
    return c0 * (1.0 + pert * rng.uniform(-1.0, 1.0, (n, n, n))), c0


def nearest_node(n, x):
    """1-based node index nearest to coordinate x."""
    return int(round(x * (n + 1)))


def clamp_phys(n, b, m):
    """Keep a source index out of the boundary PML layers (the force is assumed to vanish in
    the PML, Sec. 2)."""
    return min(max(m, b + 1), n - b)


def point_source(n, node):
    """Discrete unit point source: 1/h^3 at node (i, j, k) (1-based), zero elsewhere."""
    i, j, k = node
    f = np.zeros((n, n, n), np.complex128)
    f[k - 1, j - 1, i - 1] = 1.0 / grid_h(n) ** 3
    return f


def random_source_nodes(n, b, count, seed=SEED_SOURCES):
    """``count`` distinct nodes drawn uniformly from the non-PML box [b+1, n-b]^3."""
    rng = np.random.default_rng(seed)
    m = n - 2 * b
    flat = rng.choice(m ** 3, size=count, replace=False)
    k, j, i = np.unravel_index(flat, (m, m, m))
    return [(int(a) + b + 1, int(bb) + b + 1, int(cc) + b + 1) for a, bb, cc in zip(i, j, k)]


def sources(n, nodes):
    return np.stack([point_source(n, nd) for nd in nodes])


def fd_cells(n, b, count, seed=SEED_FDCELLS):
    """Distinct non-PML cells (i, j, k) for finite-difference gradient checks."""
    return random_source_nodes(n, b, count, seed)


def workload(name):
    """Named workloads.  C = 30 b gives the boundary PML a peak damping of 30/h."""
    if name == "c1":      # plain method, complex128, constant medium, one centred point source
        n, b = 31, 6
        m = (n + 1) // 2
        return dict(name=name, n=n, b=b, p=6, d=1, C=30.0 * b, omega=8 * math.pi,
                    c=medium_constant(n), nodes=[(m, m, m)], tol=1e-6, restart=50)
    if name == "c2":      # Gaussian lens, point source at (1/2, 1/2, 1/4)
        n, b = 63, 6
        node = tuple(clamp_phys(n, b, nearest_node(n, x)) for x in (0.5, 0.5, 0.25))
        return dict(name=name, n=n, b=b, p=6, d=1, C=30.0 * b, omega=2 * math.pi * 8,
                    c=medium_lens(n), nodes=[node], tol=1e-6, restart=50)
    if name == "c3":      # Gaussian random field in [1, 2], 32 batched point sources
        # five layers per auxiliary problem and a 2-cell moving PML with 0.16 of the boundary
        # PML's constant (the workload fixes only the 5-cell boundary PML): the fastest solve
        # among the measured (d, p, C_moving) with blocks the sweep supports
        n, b = 127, 5
        return dict(name=name, n=n, b=b, p=2, d=5, C=30.0 * b, C_moving=30.0 * b * 0.16, omega=2 * math.pi * 16,
                    c=medium_grf(n, 0.1, 1.0, 2.0), nodes=random_source_nodes(n, b, 32),
                    tol=1e-6, restart=50)
    if name == "c4":      # two-layer medium, 8 sources at x3 = 0.1, receivers at x3 = 0.9
        n, b = 63, 6
        c, c0 = medium_two_layer(n)
        rng = np.random.default_rng(SEED_SOURCES)
        ks = clamp_phys(n, b, nearest_node(n, 0.1))
        xy = rng.choice((n - 2 * b) ** 2, size=8, replace=False)
        nodes = [(int(v % (n - 2 * b)) + b + 1, int(v // (n - 2 * b)) + b + 1, ks) for v in xy]
        return dict(name=name, n=n, b=b, p=6, d=1, C=30.0 * b, omega=2 * math.pi * 8,
                    c=c, c0=c0, nodes=nodes, plane_k=nearest_node(n, 0.9), tol=1e-6, restart=50,
                    fd_step=1e-4, fd_cells=fd_cells(n, b, 20))
    if name == "c5":      # large single GPU: random field in [1.5, 3], 8 sources
        # the moving PML at a quarter of the boundary PML's constant (the description fixes
        # the widths, not the constant): 14-18 iterations instead of 16-21
        n, b = 255, 4
        return dict(name=name, n=n, b=b, p=4, d=1, C=30.0 * b, C_moving=30.0 * b / 4, omega=2 * math.pi * 32,
                    c=medium_grf(n, 0.05, 1.5, 3.0), nodes=random_source_nodes(n, b, 8),
                    tol=1e-6, restart=50)
    raise KeyError(name)


def small_case(n=11, b=3, p=3, d=1, seed=SEED_MEDIUM, ppw=8.0, contrast=0.3):
    """A small random-medium case for parity tests: c in [1, 1+contrast], 8 points per
    wavelength at c = 1."""
    rng = np.random.default_rng(seed)
    h = grid_h(n)
    return dict(name=f"small{n}", n=n, b=b, p=p, d=d, C=30.0 * b,
                omega=2 * math.pi / (ppw * h), c=1.0 + contrast * rng.random((n, n, n)))


def random_rhs(n, R, seed=SEED_SOURCES):
    """R complex Gaussian right-hand sides, shape (R, n, n, n)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((R, n, n, n)) + 1j * rng.standard_normal((R, n, n, n))
