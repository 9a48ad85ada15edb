"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module holds random-number generation and workload descriptions
only -- none of the method's arithmetic -- so both the HIP path and the oracle
can be fed the same arrays.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then the 64-bit mix
z = (z ^ z>>30) * 0xBF58476D1CE4E5B9; z = (z ^ z>>27) * 0x94D049BB133111EB;
z ^= z>>31.  A uniform double in [0, 1) is (z >> 11) * 2^-53; normals use the
Box-Muller transform of two uniforms.
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, stream=0):
    """n consecutive SplitMix64 outputs of the sequence started at
    seed * 2^32 + stream (vectorised; counter-based, so any slice can be
    regenerated independently)."""
    with np.errstate(over="ignore"):
        base = np.uint64((int(seed) << 32) + int(stream))
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = base + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed, n, lo=0.0, hi=1.0, stream=0):
    u = (splitmix64(seed, n, stream) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def normal(seed, n, stream=0):
    m = (n + 1) // 2
    u1 = uniform(seed, m, stream=stream)
    u2 = uniform(seed, m, stream=stream + 1)
    r = np.sqrt(-2.0 * np.log1p(-u1))  # 1 - u1 in (0, 1]
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def lame(E, nu):
    """Lame parameters of Young's modulus E and Poisson ratio nu."""
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


# Face bits of a Dirichlet mask: bit (face*3 + component), faces
# 0:x=0 1:x=max 2:y=0 3:y=max 4:z=0 5:z=max.
def face_bits(face, comps=(0, 1, 2)):
    b = 0
    for c in comps:
        b |= 1 << (face * 3 + c)
    return b


# Workloads shaped like the paper's tests (Section 5), synthetic stand-ins.
WORKLOADS = {
    # unit cube, 2x2x2 hexahedra (static large-strain example), P=3
    "cube8_p3": dict(n=(2, 2, 2), L=(1.0, 1.0, 1.0), P=3, E=1.0e3, nu=0.3, rho=1.0,
                     kind=4, dirichlet=face_bits(0), seed=1),
    # 16x4x4 cantilever 4x1x1, P=4, clamped at x=0
    "cantilever_p4": dict(n=(16, 4, 4), L=(4.0, 1.0, 1.0), P=4, E=1.0e3, nu=0.3, rho=1.0,
                          kind=4, dirichlet=face_bits(0), seed=2),
    # 64x64x16 block 4x4x1, P=3, impact on a rigid plane
    "impact_p3": dict(n=(64, 64, 16), L=(4.0, 4.0, 1.0), P=3, E=1.0e3, nu=0.3, rho=1.0,
                      kind=2, dirichlet=0, seed=3),
    # 16^3 unit cube, P=4, differentiable explicit run
    "adjoint_p4": dict(n=(16, 16, 16), L=(1.0, 1.0, 1.0), P=4, E=1.0e3, nu=0.3, rho=1.0,
                       kind=2, dirichlet=face_bits(0), seed=4),
    # polynomial-order sweep at ~2e7 DOF: unit cube, clamp z=0, top z=1 moved by -0.2
    "compress_p2": dict(n=(94, 94, 94), L=(1.0, 1.0, 1.0), P=2, E=1.0e3, nu=0.3, rho=1.0,
                        kind=4, dirichlet=face_bits(4) | face_bits(5), seed=5),
    "compress_p4": dict(n=(47, 47, 47), L=(1.0, 1.0, 1.0), P=4, E=1.0e3, nu=0.3, rho=1.0,
                        kind=4, dirichlet=face_bits(4) | face_bits(5), seed=5),
    "compress_p6": dict(n=(31, 31, 31), L=(1.0, 1.0, 1.0), P=6, E=1.0e3, nu=0.3, rho=1.0,
                        kind=4, dirichlet=face_bits(4) | face_bits(5), seed=5),
    "compress_p8": dict(n=(23, 23, 23), L=(1.0, 1.0, 1.0), P=8, E=1.0e3, nu=0.3, rho=1.0,
                        kind=4, dirichlet=face_bits(4) | face_bits(5), seed=5),
}


def num_nodes(n, P):
    return (n[0] * P + 1) * (n[1] * P + 1) * (n[2] * P + 1)


def random_coeffs(seed, n, P, amp, stream=0):
    """Uniform(-amp, amp) coefficient vector, SoA [3][Nn]."""
    return uniform(seed, 3 * num_nodes(n, P), -amp, amp, stream=stream)


def lognormal_lame(seed, E_count, E, nu, sigma=0.2):
    """Per-element mu, lam = median * exp(sigma z), z ~ N(0,1) independent."""
    lam0, mu0 = lame(E, nu)
    mu = mu0 * np.exp(sigma * normal(seed, E_count, stream=10))
    lam = lam0 * np.exp(sigma * normal(seed, E_count, stream=20))
    return mu, lam
