"""Test helpers: translate a workload dict to the oracle's and the library's descriptions, and map
cell orders between them (both report (level, i_x, i_y, i_z) per cell)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2408_08129_amd.cases import product_case  # noqa: F401  (re-exported for the tests)


def oracle_case(w: dict) -> O.Case:
    return O.Case(dim=w["dim"], degree=w["degree"], nbase=tuple(w["nbase"]), length=tuple(w["length"]),
                  periodic=tuple(w.get("periodic", (1, 1))), rules=list(w.get("rules", [])),
                  oro_kind=w["orography"], oro=tuple(w["oro"]), atm_kind=w["atmosphere"],
                  atm=tuple(w["atm"]), sponge=tuple(w.get("sponge", (0.0,) * 5)))


def cell_perm(prod_cells: np.ndarray, oracle_cells: np.ndarray) -> np.ndarray:
    """perm[i] = oracle index of the product's cell i."""
    index = {tuple(r): j for j, r in enumerate(oracle_cells.tolist())}
    perm = np.array([index[tuple(r)] for r in prod_cells.tolist()], dtype=np.int64)
    assert len(set(perm.tolist())) == len(perm)
    return perm


def to_product_order(a: np.ndarray, perm: np.ndarray, nloc: int) -> np.ndarray:
    """Array [..., ncell * nloc] in oracle cell order -> product cell order."""
    sh = a.shape[:-1]
    b = a.reshape(sh + (-1, nloc))[..., perm, :]
    return np.ascontiguousarray(b.reshape(sh + (-1,)))


def to_oracle_order(a: np.ndarray, perm: np.ndarray, nloc: int) -> np.ndarray:
    sh = a.shape[:-1]
    b = np.empty(sh + (len(perm), nloc), dtype=a.dtype)
    b[..., perm, :] = a.reshape(sh + (-1, nloc))
    return b.reshape(sh + (-1,))


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    """max |a - ref| / max |ref| (per field when 2D arrays are compared field by field)."""
    s = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(a - ref))) / (s if s > 0 else 1.0)


# Small meshes with 2:1 faces (used by parity tests); orography on, periodic laterally.
def tiny2d(r, oro=3, h0=120.0):
    return dict(dim=2, degree=r, nbase=(2, 1, 2), length=(1000.0, 1.0, 1000.0), periodic=(1, 1),
                rules=[(500.0, 250.0, 250.0, 0.0, 0.0)], orography=oro, oro=(h0, 300.0, 500.0, 0.0),
                atmosphere=1, atm=(1e5, 293.15, 0.01))


def tiny3d(r, oro=3, h0=120.0):
    return dict(dim=3, degree=r, nbase=(2, 2, 2), length=(1000.0, 1000.0, 1000.0), periodic=(1, 1),
                rules=[(500.0, 250.0, 250.0, 250.0, 250.0)], orography=oro,
                oro=(h0, 300.0, 500.0, 500.0), atmosphere=1, atm=(1e5, 293.15, 0.01))


def twolevel2d(r, oro=1, h0=150.0):
    return dict(dim=2, degree=r, nbase=(8, 1, 4), length=(8000.0, 1.0, 4000.0), periodic=(1, 1),
                rules=[(1000.0, 4000.0, 2500.0, 0.0, 0.0), (500.0, 4000.0, 1200.0, 0.0, 0.0)],
                orography=oro, oro=(h0, 800.0, 4000.0, 0.0), atmosphere=1, atm=(1e5, 293.15, 0.01))


def twolevel3d(r, oro=2, h0=150.0):
    return dict(dim=3, degree=r, nbase=(4, 4, 2), length=(4000.0, 4000.0, 2000.0), periodic=(1, 1),
                rules=[(1000.0, 2000.0, 1200.0, 2000.0, 1200.0), (500.0, 2000.0, 500.0, 2000.0, 500.0)],
                orography=oro, oro=(h0, 700.0, 2000.0, 2000.0), atmosphere=1, atm=(1e5, 293.15, 0.01))


def walls2d(r):
    """Lateral walls (not periodic), two levels."""
    w = twolevel2d(r)
    w["periodic"] = (0, 0)
    return w


def walls3d(r):
    """Lateral walls on all four sides (not periodic), two levels over the bell."""
    w = twolevel3d(r)
    w["periodic"] = (0, 0)
    return w
