"""Parity cases shared by the oracle fixture script and the GPU tests (problem data only:
meshes, materials, boundary kinds, initial fields, plane-wave parameters)."""
import numpy as np

from mtp_inputs import fields, meshes

DATA, PEC, PMC = meshes.DATA, meshes.PEC, meshes.PMC

CASES = {
    # config-1 workload: 2D TE, 8x8 squares split in two, P2, plane wave on all sides
    "te_planewave_p2": dict(mesh=("square", 8), p=2, q=3, m=4, T=0.5, kind=DATA, exact="pw_te"),
    "te_pmc_p1": dict(mesh=("square_pi", 4), p=1, q=2, m=2, T=0.5, kind=PMC, exact="pmc_te"),
    "te_pmc_p3": dict(mesh=("square_pi", 4), p=3, q=4, m=6, T=0.5, kind=PMC, exact="pmc_te"),
    "te_pmc_p5": dict(mesh=("square_pi", 3), p=5, q=6, m=10, T=0.4, kind=PMC, exact="pmc_te"),
    "te_pec_p4_alpha025": dict(mesh=("square", 3), p=4, q=5, m=8, T=0.3, kind=PEC, exact="pec_te", alpha=0.25),
    "te_pec_p2_eps": dict(mesh=("square", 5), p=2, q=3, m=4, T=0.4, kind=PEC, exact="pec_te", eps_split=True),
    "cav3d_p1": dict(mesh=("kuhn", 2), p=1, q=2, m=2, T=0.25, kind=PEC, exact="pec_3d"),
    "cav3d_p2": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.25, kind=PEC, exact="pec_3d"),
    "cav3d_p3": dict(mesh=("kuhn", 2), p=3, q=4, m=6, T=0.25, kind=PEC, exact="pec_3d"),
    "cav3d_p4": dict(mesh=("kuhn", 2), p=4, q=5, m=8, T=0.125, kind=PEC, exact="pec_3d"),
    # P5 in 3D (matrix-core kernels only: operator block in device memory, column-block products)
    "cav3d_p5": dict(mesh=("kuhn", 2), p=5, q=6, m=10, T=0.1, kind=PEC, exact="pec_3d"),
    "cav3d_p5_pmc_eps": dict(mesh=("kuhn", 2), p=5, q=6, m=10, T=0.1, kind=PMC, exact="pec_3d", eps_split=True),
    "cav3d_p2_pmc_eps": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.2, kind=PMC, exact="pec_3d", eps_split=True),
    "planewave3d_p2": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.2, kind=DATA, exact="pw_3d"),
    "graded3d_p3_eps": dict(mesh=("kuhn_graded", 3), p=3, q=4, m=6, T=0.06, kind=PEC, exact="pulse",
                            eps_split=True),
    "single_tri_p2": dict(mesh=("tri1", 1), p=2, q=3, m=4, T=0.5, kind=PEC, exact="pec_te"),
    "single_tet_p3": dict(mesh=("tet1", 1), p=3, q=4, m=6, T=0.3, kind=PMC, exact="pec_3d"),
    "te_pmc_p2_two_slabs": dict(mesh=("square_pi", 4), p=2, q=3, m=4, T=0.25, kind=PMC, exact="pmc_te", slabs=2),
    # sub-interval edge cases: one sub-interval (the tent top is never inverted), odd m with
    # the 4-row tiles (P3 in 3D), and first-order Taylor (q = 1: no recursion step)
    "te_pmc_p2_m1": dict(mesh=("square_pi", 4), p=2, q=3, m=1, T=0.1, kind=PMC, exact="pmc_te"),
    "cav3d_p3_m5": dict(mesh=("kuhn", 2), p=3, q=4, m=5, T=0.25, kind=PEC, exact="pec_3d"),
    "cav3d_p2_q1_m3": dict(mesh=("kuhn", 2), p=2, q=1, m=3, T=0.1, kind=PEC, exact="pec_3d"),
    # patches beyond 8 and 24 elements (the kernels' 24- and 48-element instantiations):
    # 2D fans around a centre vertex of valence 12 and 32, and a jittered Delaunay cube
    # whose vertex patches hold up to 36 tets
    "te_fan12_p3": dict(mesh=("fan", 12), p=3, q=4, m=6, T=0.2, kind=PMC, exact="pec_te"),
    "te_fan32_p2_data": dict(mesh=("fan", 32), p=2, q=3, m=4, T=0.2, kind=DATA, exact="pw_te"),
    "te_fan32_p5": dict(mesh=("fan", 32), p=5, q=6, m=10, T=0.1, kind=PEC, exact="pec_te"),
    "delaunay3d_p2": dict(mesh=("delaunay", 3), p=2, q=3, m=4, T=0.1, kind=PEC, exact="pec_3d"),
    "delaunay3d_p3_eps": dict(mesh=("delaunay", 3), p=3, q=4, m=6, T=0.1, kind=PMC, exact="pec_3d",
                              eps_split=True),
}

# P4 on the jittered Delaunay cube, whose vertex patches hold up to 36 tets (the P4 kernels'
# 36-tet class, with the operator block in device memory)
LARGE_P4_CASES = {
    "delaunay3d_p4": dict(mesh=("delaunay", 3), p=4, q=5, m=8, T=0.05, kind=PEC, exact="pec_3d"),
    "delaunay3d_p4_pmc_eps": dict(mesh=("delaunay", 3), p=4, q=5, m=8, T=0.05, kind=PMC, exact="pec_3d",
                                  eps_split=True),
    "delaunay3d_p4_rk4": dict(mesh=("delaunay", 3), p=4, q=5, m=8, T=0.05, kind=PEC, exact="pec_3d", method="rk4"),
    "ac_delaunay3d_p4": dict(mesh=("delaunay", 3), p=4, q=5, m=8, T=0.05, kind=PMC, exact="ac_pulse3",
                             system="acoustic"),
    # patches of 37-48 tets (F/R of the tent in device memory)
    "delaunay48_p4": dict(mesh=("delaunay48", 4), p=4, q=5, m=8, T=0.04, kind=PEC, exact="pec_3d"),
    "delaunay48_p4_pmc_eps": dict(mesh=("delaunay48", 4), p=4, q=5, m=8, T=0.04, kind=PMC, exact="pec_3d",
                                  eps_split=True),
    "ac_delaunay48_p4": dict(mesh=("delaunay48", 4), p=4, q=5, m=8, T=0.04, kind=PMC, exact="ac_pulse3",
                             system="acoustic"),
    "delaunay48_p4_rk4": dict(mesh=("delaunay48", 4), p=4, q=5, m=8, T=0.04, kind=PEC, exact="pec_3d",
                              method="rk4"),
    "ac_delaunay48_p4_rk4": dict(mesh=("delaunay48", 4), p=4, q=5, m=8, T=0.04, kind=PMC, exact="ac_pulse3",
                                 system="acoustic", method="rk4"),
    # P5 on the same cubes: patches of 25-36 and 37-48 tets (operator block and F/R in device memory)
    "delaunay3d_p5": dict(mesh=("delaunay", 3), p=5, q=6, m=10, T=0.02, kind=PEC, exact="pec_3d"),
    "delaunay48_p5_pmc_eps": dict(mesh=("delaunay48", 4), p=5, q=6, m=10, T=0.02, kind=PMC, exact="pec_3d",
                                  eps_split=True),
}

# the classical RK4 variant (method="rk4"): same inputs, RK4 on the tent ODE
RK4_CASES = {
    "te_planewave_p2_rk4": dict(mesh=("square", 8), p=2, q=3, m=4, T=0.5, kind=DATA, exact="pw_te", method="rk4"),
    "te_pmc_p3_rk4": dict(mesh=("square_pi", 4), p=3, q=4, m=6, T=0.5, kind=PMC, exact="pmc_te", method="rk4"),
    "cav3d_p2_rk4": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.25, kind=PEC, exact="pec_3d", method="rk4"),
    "te_pec_p2_eps_rk4": dict(mesh=("square", 5), p=2, q=3, m=4, T=0.4, kind=PEC, exact="pec_te", eps_split=True,
                              method="rk4"),
}

# the impedance-matched flux (flux="impedance") across material jumps
IMP_CASES = {
    "te_pec_p2_eps_imp": dict(mesh=("square", 5), p=2, q=3, m=4, T=0.4, kind=PEC, exact="pec_te", eps_split=True,
                              flux="impedance"),
    "cav3d_p2_pmc_eps_imp": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.2, kind=PMC, exact="pec_3d", eps_split=True,
                                 flux="impedance"),
    "graded3d_p3_eps_imp": dict(mesh=("kuhn_graded", 3), p=3, q=4, m=6, T=0.06, kind=PEC, exact="pulse",
                                eps_split=True, flux="impedance"),
    "te_planewave_p2_imp": dict(mesh=("square", 8), p=2, q=3, m=4, T=0.5, kind=DATA, exact="pw_te", flux="impedance"),
}

# linear acoustics (system="acoustic"): kind PMC = rigid wall, PEC = pressure release;
# eps / mu hold (kappa, rho)
AC_CASES = {
    "ac2d_rigid_p3": dict(mesh=("square", 4), p=3, q=4, m=6, T=0.4, kind=PMC, exact="ac_cav2", system="acoustic"),
    "ac2d_planewave_p2": dict(mesh=("square", 6), p=2, q=3, m=4, T=0.4, kind=DATA, exact="ac_pw2", system="acoustic"),
    "ac3d_rigid_p2": dict(mesh=("kuhn", 2), p=2, q=3, m=4, T=0.25, kind=PMC, exact="ac_cav3", system="acoustic"),
    "ac3d_release_eps_p3": dict(mesh=("kuhn", 2), p=3, q=4, m=6, T=0.2, kind=PEC, exact="ac_pulse3",
                                eps_split=True, system="acoustic"),
    "ac3d_graded_imp_p4": dict(mesh=("kuhn_graded", 3), p=4, q=5, m=8, T=0.05, kind=PMC, exact="ac_pulse3",
                               eps_split=True, system="acoustic", flux="impedance"),
}


# linear acoustics under the classical RK4 variant (FP64 matrix-core kernel)
AC_RK4_CASES = {
    "ac2d_rigid_p3_rk4": dict(mesh=("square", 4), p=3, q=4, m=6, T=0.4, kind=PMC, exact="ac_cav2", system="acoustic",
                              method="rk4"),
    "ac3d_release_eps_p3_rk4": dict(mesh=("kuhn", 2), p=3, q=4, m=6, T=0.2, kind=PEC, exact="ac_pulse3",
                                    eps_split=True, system="acoustic", method="rk4"),
}


# Curved cases: the disk with quadratic boundary triangles (oracle/curved.py, weight-adjusted
# scheme), against the circular-cavity TE mode's initial data.
CURVED_CASES = {
    "disk_curved_p2": dict(mesh=("disk", 3), p=2, q=3, m=4, T=0.2, kind=PEC, exact="disk_te", curved=True),
    "disk_curved_p3_pmc": dict(mesh=("disk", 2), p=3, q=4, m=6, T=0.15, kind=PMC, exact="disk_te", curved=True),
    "disk_curved_p4_eps": dict(mesh=("disk", 2), p=4, q=5, m=8, T=0.1, kind=PEC, exact="disk_te", curved=True,
                               eps_split=True),
    "disk_curved_p1_two_slabs": dict(mesh=("disk", 3), p=1, q=2, m=2, T=0.1, kind=PEC, exact="disk_te",
                                     curved=True, slabs=2),
}

# The colour pitching rule (rule="colour"): the same problems pitched by colour turns
# instead of the minimum vertex: wide layers on the irregular disk and fan, the Kuhn
# cube's eight colours, data faces, and the curved disk.
COLOUR_CASES = {
    "disk_colour_p2": dict(mesh=("disk", 4), p=2, q=3, m=4, T=0.2, kind=PEC, exact="disk_te", rule="colour"),
    "te_fan32_p3_colour": dict(mesh=("fan", 32), p=3, q=4, m=6, T=0.1, kind=PMC, exact="pec_te", rule="colour"),
    "cav3d_p3_colour": dict(mesh=("kuhn", 2), p=3, q=4, m=6, T=0.25, kind=PEC, exact="pec_3d", rule="colour",
                            eps_split=True),
    "te_planewave_p2_colour": dict(mesh=("square", 8), p=2, q=3, m=4, T=0.5, kind=DATA, exact="pw_te",
                                   rule="colour"),
    "disk_curved_p3_colour": dict(mesh=("disk", 3), p=3, q=4, m=6, T=0.15, kind=PMC, exact="disk_te", curved=True,
                                  rule="colour", slabs=2),
}


def build_mesh(spec):
    kind, n = spec
    if kind == "square":
        return meshes.square_tri(n)
    if kind == "square_pi":
        return meshes.square_tri(n, length=np.pi)
    if kind == "kuhn":
        return meshes.cube_kuhn(n)
    if kind == "kuhn_graded":
        return meshes.cube_kuhn(n, axis_map=lambda g: 0.25 * g + 0.75 * g * g)
    if kind == "fan":
        return meshes.fan_disk(n)
    if kind == "delaunay":   # 4^3 lattice on the unit cube, jitter 0.3 h, 179 tets, patches up to 36
        return meshes.graded_delaunay_cube(n=n, a=1.0, jitter=0.3, seed=3)
    if kind == "delaunay48":   # 5^3 lattice, jitter 0.5 h, 420 tets, two patches above 36 (the largest 48)
        return meshes.graded_delaunay_cube(n=n, a=1.0, jitter=0.5, seed=180)
    if kind == "disk":
        return meshes.disk_tri(n)
    if kind == "tri1":
        return {"coords": np.array([[0.1, 0.0], [1.0, 0.2], [0.3, 0.9]]), "cells": np.array([[0, 1, 2]], np.int32)}
    if kind == "tet1":
        return {"coords": np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.2, 0.8]]),
                "cells": np.array([[0, 1, 2, 3]], np.int32)}
    raise ValueError(kind)


def exact_solution(name):
    return {"pw_te": fields.PlaneWaveTE(direction=(1.0, 1.0), k=2 * np.pi),
            "pmc_te": fields.CavityTE_PMC(),
            "pec_te": fields.CavityTE_PEC(),
            "pec_3d": fields.Cavity3D_PEC(),
            "pw_3d": fields.PlaneWave3D(direction=(1.0, 0.5, 0.25), k=np.pi, amp_e=(0.0, 1.0, -1.0), phase=0.3),
            "pulse": fields.GaussianPulse3D(seed=11030),
            "ac_cav2": fields.AcousticCavity(2),
            "ac_cav3": fields.AcousticCavity(3),
            "ac_pw2": fields.AcousticPlaneWave(direction=(1.0, 0.6), k=2 * np.pi, phase=0.2),
            "ac_pulse3": fields.AcousticPulse(3),
            "disk_te": fields.CircularCavityTE()}[name]


def planewave_params(ex, dim):
    """(amp, kvec, omega, phase) of a plane-wave exact solution for the C interface."""
    if hasattr(ex, "avec"):        # acoustics: amplitude of (p, v)
        amp = ex.avec
    elif dim == 2:
        amp = np.array([-ex.d[1] * ex.amp, ex.d[0] * ex.amp, ex.amp * np.sqrt(ex.eps / ex.mu)])
    else:
        amp = np.concatenate([ex.aE, ex.aH])
    return amp, ex.k * ex.d, ex.omega, ex.phase


def setup(name):
    c = dict(CASES.get(name) or RK4_CASES.get(name) or IMP_CASES.get(name) or CURVED_CASES.get(name)
             or COLOUR_CASES.get(name) or LARGE_P4_CASES.get(name) or AC_RK4_CASES.get(name) or AC_CASES[name])
    c.setdefault("curved", False)
    c.setdefault("rule", "min_vertex")
    c.setdefault("system", "maxwell")
    c.setdefault("method", "sat")
    c.setdefault("flux", "penalty")
    c.setdefault("alpha", 0.5)
    c.setdefault("slabs", 1)
    c.setdefault("eps_split", False)
    mm = build_mesh(c["mesh"])
    dim = mm["coords"].shape[1]
    ne = len(mm["cells"])
    if c["eps_split"]:
        eps, mu = meshes.materials_split(mm)
    else:
        eps, mu = np.ones(ne), np.ones(ne)
    ex = exact_solution(c["exact"])
    if c["curved"]:
        mm["geo"] = meshes.p2_geometry(mm, on_circle=1.0)
        u0 = ex.u(meshes.equispaced_nodes_p2(mm["geo"], c["p"]), 0.0)
    else:
        u0 = ex.u(meshes.equispaced_nodes(mm, c["p"]), 0.0)
    return c, mm, dim, eps, mu, meshes.uniform_bc(ne, dim, c["kind"]), ex, u0
