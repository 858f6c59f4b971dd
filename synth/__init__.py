"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers and lays them out as plain tables; it
contains none of the solver's arithmetic.  Both sides receive the same tables
(mode tables for right-hand sides, instance lists for batches, random vectors)
and evaluate them with their own code.

Random-field right-hand side (used for the annulus, batched and learned-smoother
workloads): f(x, y) = sum_m a_m sin(pi (k_m x + l_m y) + phi_m), with the 1/8
normalisation folded into a_m.  A mode table has one row per mode:
(a, k, l, phi) in 2D and (a, k, l, m, phi) in 3D.
"""
import math

import numpy as np

N_FIELD_MODES = 64


def random_field_modes(seed, n_modes=N_FIELD_MODES):
    """Mode table (n_modes x 4) of the seeded smooth random field.

    Draw order: a ~ N(0,1), k ~ U{1..8}, l ~ U{1..8}, phi ~ U[0, 2 pi), each as
    a block of n_modes values; a is then scaled by 1/8.
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n_modes)
    k = rng.integers(1, 9, size=n_modes)
    l = rng.integers(1, 9, size=n_modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return np.column_stack([a / 8.0, k, l, phi]).astype(np.float64)


def manufactured_sine_modes_2d():
    """Mode table of f = 2 pi^2 sin(pi x) sin(pi y) (exact u = sin pi x sin pi y).

    Uses sin A sin B = (sin(A - B + pi/2) - sin(A + B + pi/2)) / 2.
    """
    c = math.pi ** 2
    h = 0.5 * math.pi
    return np.array([[c, 1.0, -1.0, h], [-c, 1.0, 1.0, h]], dtype=np.float64)


def poisson_2d_sine_modes(k=1):
    """Mode table of f = 2 (2 k pi)^2 sin(2 k pi x) sin(2 k pi y), exact
    u = sin(2 k pi x) sin(2 k pi y): the 2D Poisson model problem of Section 4.2."""
    c = (2.0 * k * math.pi) ** 2
    h = 0.5 * math.pi
    return np.array([[c, 2.0 * k, -2.0 * k, h], [-c, 2.0 * k, 2.0 * k, h]], dtype=np.float64)


def manufactured_sine_modes_3d():
    """Mode table of f = 3 pi^2 sin(pi x) sin(pi y) sin(pi z).

    Uses 4 sin A sin B sin C = sin(A+B-C) + sin(A-B+C) + sin(-A+B+C) - sin(A+B+C).
    """
    c = 0.75 * math.pi ** 2
    return np.array([[c, 1, 1, -1, 0.0], [c, 1, -1, 1, 0.0], [c, -1, 1, 1, 0.0],
                     [-c, 1, 1, 1, 0.0]], dtype=np.float64)


def random_vector(n, seed):
    """Seeded N(0,1) vector of length n (float64)."""
    return np.random.default_rng(seed).standard_normal(n)


BATCH_BASES = (4, 5, 6, 7)


def batch_element_counts():
    """Elements per direction allowed in a batch: m * 2^j in [32, 512], m in 4..7."""
    out = set()
    for m in BATCH_BASES:
        v = m
        while v <= 512:
            if v >= 32:
                out.add(v)
            v *= 2
    return sorted(out)


def batch_instances(count=96, seed=4):
    """Seeded list of batch instances: (n_el, degree, geometry, rhs_seed).

    Draw order: n_el[count] uniform over batch_element_counts(), degree[count]
    uniform over {2..5}, geometry[count] Bernoulli(1/2) (0 square, 1 annulus).
    """
    rng = np.random.default_rng(seed)
    choices = np.array(batch_element_counts())
    n_el = choices[rng.integers(0, len(choices), size=count)]
    deg = rng.integers(2, 6, size=count)
    geom = rng.integers(0, 2, size=count)
    return [(int(n_el[i]), int(deg[i]), int(geom[i]), 4000 + i) for i in range(count)]
