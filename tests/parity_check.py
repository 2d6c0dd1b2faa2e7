"""Parity measures of a GPU field against the oracle's (reading A18 of the discrete definition).

Both are taken over the device cells only (the planes between the contacts): the metal planes
hold fixed contact potentials on both sides and would only inflate the norms.

* rel_dev: ||a - b||_2 / ||b||_2 over device cells;
* max_dev: max |a - b| / max |b| over device cells (a per-cell bound, so that an error
  confined to a few cells cannot hide inside the L2 norm of a large grid).
"""
import numpy as np


def device(spec, x):
    kb, kt = spec.device_range()
    return np.asarray(x)[kb:kt]


def rel_dev(spec, a, b):
    da, db = device(spec, a), device(spec, b)
    nb = np.linalg.norm(db)
    return float(np.linalg.norm(da - db) / (nb if nb > 0 else 1.0))


def max_dev(spec, a, b):
    da, db = device(spec, a), device(spec, b)
    mb = np.abs(db).max()
    return float(np.abs(da - db).max() / (mb if mb > 0 else 1.0))


def check(spec, a, b, tol, what=""):
    """Assert both measures within tol; returns them for printing."""
    r, m = rel_dev(spec, a, b), max_dev(spec, a, b)
    assert r <= tol, f"{what}: relative L2 over device cells {r:.3e} > {tol:.1e}"
    assert m <= tol, f"{what}: max-abs over device cells {m:.3e} (of max |oracle|) > {tol:.1e}"
    return r, m


def worst(spec, a, b):
    """The larger of the two measures (for tests that print one figure per field)."""
    return max(rel_dev(spec, a, b), max_dev(spec, a, b))
