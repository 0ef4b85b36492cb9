"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws seeded random
numbers and evaluates the synthetic fields that define the workloads
(random vectors, a spherical-harmonic temperature, the viscosity and density
profiles of the shell configurations).  Everything is FP64 numpy.
"""
import numpy as np
from scipy.special import lpmv

R_IN, R_OUT = 0.55, 1.0


def uniform(seed, n, lo=-1.0, hi=1.0):
    """n values uniform in [lo, hi) from numpy's default generator."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def normal(seed, n):
    return np.random.default_rng(seed).standard_normal(n)


class SHField:
    """S(x) = sum_{l<=lmax, |m|<=l} a_lm Y_lm(x/|x|) cos(pi c_lm (r - r_in)/(r_out - r_in))

    with real spherical harmonics, a_lm ~ N(0,1)/(l+1) and c_lm in {0,1,2},
    all drawn from ``seed``.  ``temperature`` maps S to [0, 1] with a bound
    taken on a fixed seeded sample of the shell, so the field does not
    depend on the mesh it is evaluated on.
    """

    def __init__(self, seed, lmax=8, r_in=R_IN, r_out=R_OUT):
        rng = np.random.default_rng(seed)
        self.terms = []
        for l in range(lmax + 1):
            for m in range(-l, l + 1):
                self.terms.append((l, m, rng.standard_normal() / (l + 1), int(rng.integers(0, 3))))
        self.r_in, self.r_out = r_in, r_out
        srng = np.random.default_rng(seed + 1000)
        d = srng.standard_normal((4096, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = srng.uniform(r_in, r_out, 4096)
        self.smax = 1.05 * np.abs(self.raw(d * r[:, None])).max()

    def raw(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64)
        r = np.linalg.norm(xyz, axis=1)
        ct = np.clip(xyz[:, 2] / r, -1.0, 1.0)
        ph = np.arctan2(xyz[:, 1], xyz[:, 0])
        s = np.zeros(len(xyz))
        for (l, m, a, c) in self.terms:
            ang = np.cos(m * ph) if m >= 0 else np.sin(-m * ph)
            s += a * lpmv(abs(m), l, ct) * ang * np.cos(np.pi * c * (r - self.r_in) / (self.r_out - self.r_in))
        return s

    def temperature(self, xyz):
        return np.clip(0.5 + 0.5 * self.raw(xyz) / self.smax, 0.0, 1.0)

    def temperature_torch(self, xyz):
        """Same field for a (n, 3) float64 torch tensor, evaluated where the
        tensor lives (associated Legendre functions by the standard
        three-term recurrence, Condon-Shortley phase as scipy's lpmv)."""
        import torch
        r = torch.linalg.norm(xyz, dim=1)
        ct = torch.clamp(xyz[:, 2] / r, -1.0, 1.0)
        st = torch.sqrt(torch.clamp(1.0 - ct * ct, min=0.0))
        ph = torch.atan2(xyz[:, 1], xyz[:, 0])
        lmax = max(l for (l, _, _, _) in self.terms)
        P = {}
        for m in range(lmax + 1):
            pmm = torch.ones_like(ct)
            fact = 1.0
            for _ in range(m):
                pmm = -pmm * fact * st
                fact += 2.0
            P[(m, m)] = pmm
            if m + 1 <= lmax:
                P[(m + 1, m)] = ct * (2 * m + 1) * pmm
            for l in range(m + 2, lmax + 1):
                P[(l, m)] = ((2 * l - 1) * ct * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
        s = torch.zeros_like(ct)
        for (l, m, a, c) in self.terms:
            ang = torch.cos(m * ph) if m >= 0 else torch.sin(-m * ph)
            s += a * P[(l, abs(m))] * ang * torch.cos(np.pi * c * (r - self.r_in) / (self.r_out - self.r_in))
        return torch.clamp(0.5 + 0.5 * s / self.smax, 0.0, 1.0)


def viscosity_contrast(T, contrast=1e4):
    """eta = exp(ln(contrast) (0.5 - T)), in [contrast^-1/2, contrast^1/2] for T in [0,1]."""
    return np.exp(np.log(contrast) * (0.5 - np.asarray(T)))


def viscosity_1e6(xyz, T, seed=3, contrast=1e6, r_in=R_IN, r_out=R_OUT):
    """eta = 100^((r_out - r)/(r_out - r_in)) * exp(a (0.5 - T)) * (100 in a slab
    {r >= 0.75, angle(x, c) <= 15 deg} around a seeded direction c, else 1),
    with the temperature exponent a >= 0 chosen so that max/min of eta over
    the given points is `contrast` (a depth factor of 100 and the slab alone
    reach only about 1.3e3).  log eta is affine in a, so its spread is a
    convex piecewise-linear function of a, found by bisection."""
    xyz = np.asarray(xyz, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    r = np.linalg.norm(xyz, axis=1)
    c = np.random.default_rng(seed).standard_normal(3)
    c /= np.linalg.norm(c)
    cosang = (xyz @ c) / r
    slab = (r >= 0.75) & (cosang >= np.cos(np.deg2rad(15.0)))
    b = np.log(100.0) * (r_out - r) / (r_out - r_in) + np.where(slab, np.log(100.0), 0.0)
    spread = lambda a: np.ptp(b + a * (0.5 - T))
    target = np.log(contrast)
    lo, hi = 0.0, 1.0
    while spread(hi) < target:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if spread(mid) < target else (lo, mid)
    return np.exp(b + 0.5 * (lo + hi) * (0.5 - T))


def ln_density(xyz):
    """ln rho with rho = exp(0.5 (1 - r))."""
    return 0.5 * (1.0 - np.linalg.norm(np.asarray(xyz), axis=1))


def smooth_vector_field(seed, xyz, k=3):
    """A seeded smooth 3-vector field sum of a few sines, for sampled checks."""
    rng = np.random.default_rng(seed)
    xyz = np.asarray(xyz, dtype=np.float64)
    out = np.zeros((len(xyz), 3))
    for _ in range(k):
        w = rng.normal(0.0, 3.0, 3)
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.uniform(-1, 1, 3)
        out += np.sin(xyz @ w + ph)[:, None] * a[None, :]
    return out


def smooth_vector_field_torch(seed, xyz, k=3):
    """smooth_vector_field for an (n, 3) float64 torch tensor, evaluated where
    the tensor lives; returned component-major (3 n), as the solver stores
    velocities."""
    import torch
    rng = np.random.default_rng(seed)
    out = torch.zeros(3, xyz.shape[0], dtype=torch.float64, device=xyz.device)
    for _ in range(k):
        w = rng.normal(0.0, 3.0, 3)
        ph = rng.uniform(0, 2 * np.pi)
        a = rng.uniform(-1, 1, 3)
        s = torch.sin(float(w[0]) * xyz[:, 0] + float(w[1]) * xyz[:, 1] + float(w[2]) * xyz[:, 2] + ph)
        for c in range(3):
            out[c] += float(a[c]) * s
    return out.reshape(-1)


def plate_velocity(seed, xyz, n_plates=6, scale=0.5):
    """Synthetic tangential surface velocity: the sphere split into
    ``n_plates`` Voronoi plates around seeded centres, each rotating rigidly
    about its own seeded Euler pole, u = scale * omega_k x X.  Stands in for a
    plate reconstruction (the factor 1/2 as in the paper's model setup)."""
    rng = np.random.default_rng(seed)
    xyz = np.asarray(xyz, dtype=np.float64)
    centres = rng.normal(size=(n_plates, 3))
    centres /= np.linalg.norm(centres, axis=1)[:, None]
    poles = rng.normal(0.0, 1.0, size=(n_plates, 3))
    r = np.linalg.norm(xyz, axis=1)
    unit = xyz / np.where(r > 0, r, 1.0)[:, None]
    plate = np.argmax(unit @ centres.T, axis=1)
    return scale * np.cross(poles[plate], xyz)


def base_viscosity_profile(n=65, r_in=R_IN, r_out=R_OUT):
    """Synthetic radial base viscosity eta_base on a uniform grid of n radii:
    log-linear through a stiff lower mantle, a weak asthenosphere and a stiff
    lithosphere.  Stands in for the profile the paper shows only as a figure."""
    r = np.linspace(r_in, r_out, n)
    knots = np.array([r_in, 0.85, 0.88, 0.95, 0.97, r_out])
    log10 = np.array([1.5, 1.0, -1.0, -1.0, 2.0, 2.0])
    return 10.0 ** np.interp(r, knots, log10)


def splitmix64(state, n):
    """The first n 64-bit outputs of the splitmix64 generator (Steele, Lea and
    Flood, OOPSLA 2014) started from `state`: the state advances by the
    golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state
    passed through the generator's two xor-shift-multiply rounds and a final
    xor-shift."""
    M = (1 << 64) - 1
    out = []
    st = state & M
    for _ in range(n):
        st = (st + 0x9E3779B97F4A7C15) & M
        z = st
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        out.append(z ^ (z >> 31))
    return out


def splitmix64_uniform(state, n):
    """n values uniform in [-1, 1) from splitmix64: the top 53 bits of each
    output give the double.  Tests use it to reproduce a start vector the
    library draws with the same published generator."""
    return np.array([(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0 for z in splitmix64(state, n)])
