"""Named synthetic workloads (plain data).

Each entry describes a problem: the logical box, the base grid, refinement rules (Section 3.1 /
Fig. 1: finer cells near the orography), the orography, the atmosphere, the wind, the time step and
the number of steps.  The orographies follow Section 3.1, Eq. (3) (bell) and its 2D / Gaussian
variants; the stratified atmosphere is that of Eq. (4)-(5) with N = 0.01 1/s.
"""
from __future__ import annotations

ORO_FLAT, ORO_AGNESI, ORO_BELL, ORO_GAUSS_HILL, ORO_GAUSS_RIDGE = range(5)
ATM_ISOTHERMAL, ATM_STRATIFIED = range(2)

STRAT = (1.0e5, 293.15, 0.01)
# absorbing layers of the bell-hill case: (top depth, top rate, side width, side rate, u_ref)
BELL_LAYERS = (6000.0, 0.05, 10000.0, 0.05, 10.0)

WORKLOADS = {
    # 2D slice, degree 2, conforming 32 x 16 quads on 20 km x 10 km, isothermal 250 K,
    # Agnesi hill h = 1 m, a = 1 km, u = 10 m/s, dt = 1 s, 10 steps.
    "slice2d_r2_conforming": dict(
        dim=2, degree=2, nbase=(32, 1, 16), length=(20000.0, 1.0, 10000.0), periodic=(1, 1),
        rules=[], orography=ORO_AGNESI, oro=(1.0, 1000.0, 10000.0, 0.0),
        atmosphere=ATM_ISOTHERMAL, atm=(1.0e5, 250.0, 0.0), ubar=10.0, dt=1.0, steps=10),
    # 2D slice, degree 4, 64 x 32 base quads, two 2:1 levels in the lowest 2 km (hanging faces of
    # both orientations): 3200 cells; Agnesi h = 400 m, stratified N = 0.01, u = 10 m/s.
    "slice2d_r4_twolevel": dict(
        dim=2, degree=4, nbase=(64, 1, 32), length=(20000.0, 1.0, 10000.0), periodic=(1, 1),
        rules=[(2000.0, 10000.0, 5000.0, 0.0, 0.0), (1000.0, 10000.0, 2500.0, 0.0, 0.0)],
        orography=ORO_AGNESI, oro=(400.0, 1000.0, 10000.0, 0.0), atmosphere=ATM_STRATIFIED,
        atm=STRAT, ubar=10.0, dt=0.15, steps=200),
    # 3D box 40 x 40 x 20 km, degree 4, 64 x 64 x 32 base hexahedra, one level below 3 km:
    # 274,432 cells, 171.5 M DoFs; Gaussian hill h = 400 m, sigma = 2 km.
    "box3d_r4_hill": dict(
        dim=3, degree=4, nbase=(64, 64, 32), length=(40000.0, 40000.0, 20000.0), periodic=(1, 1),
        rules=[(3000.0, 0.0, -1.0, 0.0, -1.0)], orography=ORO_GAUSS_HILL,
        oro=(400.0, 2000.0, 20000.0, 20000.0), atmosphere=ATM_STRATIFIED, atm=STRAT, ubar=10.0,
        dt=0.6, steps=50),
    # Large 3D case: 128^3 base hexahedra, degree 4, two levels near a Gaussian ridge (h = 1 km,
    # half-width 5 km): 2,183,168 cells, 1.36e9 DoFs.
    "box3d_r4_ridge_large": dict(
        dim=3, degree=4, nbase=(128, 128, 128), length=(128000.0, 128000.0, 32000.0),
        periodic=(1, 1),
        rules=[(2000.0, 64000.0, 2500.0, 0.0, -1.0), (1000.0, 64000.0, 1250.0, 0.0, -1.0)],
        orography=ORO_GAUSS_RIDGE, oro=(1000.0, 5000.0, 64000.0, 0.0),
        atmosphere=ATM_STRATIFIED, atm=STRAT, ubar=10.0, dt=0.4, steps=20),
    # The 3D bell-hill test of Section 3.1: 60 x 40 x 16 km, bell of Eq. (3) with h_c = 400 m,
    # a_c = 1 km at (30, 20) km, stratified N = 0.01, u = 10 m/s, degree 4, dt = 2 s, one hour.
    # Non-reflecting top and sides as absorbing layers (6 km below the lid, 10 km along each
    # periodic side, rates 0.05 1/s, towards the background wind).  Run with the enthalpy split
    # of the implicit energy flux and without the pressure-jump penalty (stable for long runs in
    # a stratified atmosphere).  Uniform: 60 x 40 x 16 cells of 1 km (250 m between nodes),
    # 38,400 cells.
    "bell3d_r4_uniform": dict(
        dim=3, degree=4, nbase=(60, 40, 16), length=(60000.0, 40000.0, 16000.0), periodic=(1, 1),
        rules=[], orography=ORO_BELL, oro=(400.0, 1000.0, 30000.0, 20000.0),
        atmosphere=ATM_STRATIFIED, atm=STRAT, ubar=10.0, dt=2.0, steps=1800,
        sponge=BELL_LAYERS, enthalpy_split=1, penalty_beta=0.0),
    # Non-conforming: 15 x 10 x 4 base cells of 4 km, 2 km cells over the lowest 4 km, 1 km cells
    # (the uniform mesh's size) over the lowest 2 km within 10 km (x) and 4 km (y) of the hill:
    # 450 + 1160 + 320 = 1930 cells (the paper's mesh of 1958 cells is shown only as a figure).
    "bell3d_r4_nonconforming": dict(
        dim=3, degree=4, nbase=(15, 10, 4), length=(60000.0, 40000.0, 16000.0), periodic=(1, 1),
        rules=[(4000.0, 0.0, -1.0, 0.0, -1.0), (2000.0, 30000.0, 10000.0, 20000.0, 4000.0)],
        orography=ORO_BELL, oro=(400.0, 1000.0, 30000.0, 20000.0), atmosphere=ATM_STRATIFIED,
        atm=STRAT, ubar=10.0, dt=2.0, steps=1800, sponge=BELL_LAYERS, enthalpy_split=1,
        penalty_beta=0.0),
}


def product_case(w: dict):
    """Workload dict -> the binding's Case (the problem description passed to dg_setup)."""
    from . import Case
    return Case(dim=w["dim"], nbase=tuple(w["nbase"]), length=tuple(w["length"]),
                periodic=tuple(w.get("periodic", (1, 1))), rules=list(w.get("rules", [])),
                orography=w["orography"], oro=tuple(w["oro"]), atmosphere=w["atmosphere"],
                atm=tuple(w["atm"]), sponge=tuple(w.get("sponge", (0.0,) * 5)))


def column_sample(w: dict, nx: int, ny: int) -> dict:
    """The same workload restricted to nx (x ny) base columns around the orography: full height,
    same cell sizes and refinement rules, the hill centred in the sample."""
    out = dict(w)
    nb = list(w["nbase"])
    L = list(w["length"])
    dx = L[0] / nb[0]
    dy = L[1] / nb[1]
    cx = w["oro"][2]
    cy = w["oro"][3]
    nb[0] = nx
    L[0] = nx * dx
    if w["dim"] == 3:
        nb[1] = ny
        L[1] = ny * dy
    out["nbase"] = tuple(nb)
    out["length"] = tuple(L)
    sx = L[0] / 2.0 - cx
    sy = (L[1] / 2.0 - cy) if w["dim"] == 3 else 0.0
    out["rules"] = [(r[0], r[1] + sx, r[2], r[3] + sy, r[4]) for r in w["rules"]]
    o = list(w["oro"])
    o[2] += sx
    if w["dim"] == 3:
        o[3] += sy
    out["oro"] = tuple(o)
    return out
