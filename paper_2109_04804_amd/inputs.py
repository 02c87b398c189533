"""Seeded synthetic inputs for the workloads (shared by tests, smoke and bench).

This module holds no arithmetic of the numerical method: it places nodes on a
uniform Cartesian mesh from a given set of 1-D reference nodes, evaluates
closed-form initial conditions there, and draws seeded random fields.  The
caller passes the 1-D reference nodes in.

Workloads (all periodic):
  advection_sine   u0 = sin(2 pi x) on [0, 1]                      (1-D advection)
  burgers          u0 = 0.5 + 0.25 sin(x + y) + seeded Fourier noise on [0, 2pi]^2
                   noise: modes k in Z^2 with 0 < |k|^2 <= 16 (48 modes),
                   a_k, b_k ~ U(-1, 1) from numpy default_rng(seed) in
                   lexicographic (kx, ky) order, sum a cos(k.x) + b sin(k.x),
                   rescaled to max |noise| = 1e-3 over the nodes given
  isentropic_vortex  rho_inf = p_inf = 1, strength beta, centre (xc, yc),
                   background velocity M sqrt(gamma) (1, 1)/sqrt(2),
                   minimum-image distance on the periodic box
  taylor_green     rho = 1, v = (sin x cos y cos z, -cos x sin y cos z, 0),
                   p = rho/gamma + rho eps^2/16 (cos 2x + cos 2y)(cos 2z + 2)
  density_wave     rho = 1 + 0.3 sin(pi sum_m (x_m - a t)), v = a, p = 1 (on [-1, 1]^d)

Conserved Euler variables use E = p/(gamma - 1) + eps^2/2 rho |v|^2.
"""
import numpy as np

DEFAULT_SEED = 2109


def node_coords(dim, nelem, length, origin, xi):
    """Physical coordinates of every node: list of `dim` arrays shaped (nE, (N+1)^dim).

    Elements are lexicographic with x fastest; node = i + (N+1)(j + (N+1)k)."""
    xi = np.asarray(xi, dtype=np.float64)
    npn = len(xi)
    nelem = [int(n) for n in nelem[:dim]]
    egrid = tuple(reversed(nelem))
    out = []
    for m in range(dim):
        n = nelem[m]
        h = float(length[m]) / n
        xc = float(origin[m]) + h * (np.arange(n) + 0.5)
        eshape = [1] * dim
        eshape[dim - 1 - m] = n
        nshape = [1] * dim
        nshape[dim - 1 - m] = npn
        x = xc.reshape(eshape + [1] * dim) + 0.5 * h * xi.reshape([1] * dim + nshape)
        x = np.broadcast_to(x, egrid + (npn,) * dim)
        out.append(np.ascontiguousarray(x).reshape(int(np.prod(nelem)), npn ** dim))
    return out


def euler_conserved(rho, vel, p, gamma, eps):
    """Stack (rho, rho v, E) into shape (nE, d+2, nnode)."""
    v2 = sum(v * v for v in vel)
    E = p / (gamma - 1.0) + 0.5 * eps ** 2 * rho * v2
    return np.stack([rho] + [rho * v for v in vel] + [E], axis=1)


def advection_sine(x, t=0.0, a=1.0):
    return np.sin(2.0 * np.pi * (x - a * t))[:, None, :]


def burgers_noise_modes(seed=DEFAULT_SEED):
    modes = [(kx, ky) for kx in range(-4, 5) for ky in range(-4, 5) if 0 < kx * kx + ky * ky <= 16]
    rng = np.random.default_rng(seed)
    ab = rng.uniform(-1.0, 1.0, size=(len(modes), 2))
    return modes, ab


def burgers(x, y, seed=DEFAULT_SEED, amp=1e-3):
    modes, ab = burgers_noise_modes(seed)
    noise = np.zeros_like(x)
    for (kx, ky), (a, b) in zip(modes, ab):
        ph = kx * x + ky * y
        noise += a * np.cos(ph) + b * np.sin(ph)
    noise *= amp / np.abs(noise).max()
    return (0.5 + 0.25 * np.sin(x + y) + noise)[:, None, :]


def vortex_params(seed=DEFAULT_SEED, centre_range=(3.0, 7.0), beta=None, beta_range=(3.0, 7.0)):
    """Seeded vortex centre (and strength when beta is None)."""
    rng = np.random.default_rng(seed)
    xc, yc = rng.uniform(centre_range[0], centre_range[1], size=2)
    b = float(beta) if beta is not None else float(rng.uniform(beta_range[0], beta_range[1]))
    return float(xc), float(yc), b


def isentropic_vortex(x, y, xc, yc, beta=5.0, mach=0.5, gamma=1.4, eps=1.0, box=10.0, t=0.0):
    u_inf = mach * np.sqrt(gamma) / np.sqrt(2.0)
    cx = xc + u_inf * t
    cy = yc + u_inf * t
    dx = (x - cx + 0.5 * box) % box - 0.5 * box
    dy = (y - cy + 0.5 * box) % box - 0.5 * box
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2.0 * np.pi) * dy * f
    dv = beta / (2.0 * np.pi) * dx * f
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * np.pi ** 2) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return euler_conserved(rho, [u_inf + du, u_inf + dv], p, gamma, eps)


def taylor_green(x, y, z, gamma=1.4, eps=0.1):
    rho = np.ones_like(x)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = rho / gamma + rho * eps ** 2 / 16.0 * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return euler_conserved(rho, [u, v, w], p, gamma, eps)


def density_wave(coords, a=0.3, t=0.0, gamma=1.4, eps=1.0):
    """rho = 1 + 0.3 sin(pi sum_m (x_m - a t)), v = (a, .., a), p = 1.

    The paper writes sin(pi (x - a t)) with vector x; the scalar argument is
    read as the sum over directions (a plane wave along (1, .., 1))."""
    s = sum(c - a * t for c in coords)
    rho = 1.0 + 0.3 * np.sin(np.pi * s)
    vel = [np.full_like(rho, a) for _ in coords]
    p = np.ones_like(rho)
    return euler_conserved(rho, vel, p, gamma, eps)


def random_field(shape, seed, scale=1.0, offset=0.0):
    rng = np.random.default_rng(seed)
    return offset + scale * rng.standard_normal(shape)
