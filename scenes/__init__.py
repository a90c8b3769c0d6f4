"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds inputs: trivariate B-spline / NURBS patches (knots,
control points, scalar coefficients), piecewise-linear transfer functions and
pinhole cameras.  It holds none of the renderer's arithmetic (no basis
evaluation of its own, no inversion, no quadrature); the one place that needs
a spline's Jacobian (the twisted bar's det-J field) and the knot insertion of
the NURBS annulus call scipy's B-spline routines.
"""
from .configs import (Patch, Scene, Camera, TransferFunction, make_config, make_degenerate, make_edge_lattice,
                      make_annulus, make_mixed_degree, with_displacement,
                      open_uniform_knots, greville, affine_patch,
                      camera_from_angles, random_tf)

__all__ = ["Patch", "Scene", "Camera", "TransferFunction", "make_config", "make_degenerate", "make_edge_lattice", "make_annulus", "make_mixed_degree", "with_displacement",
           "open_uniform_knots", "greville", "affine_patch",
           "camera_from_angles", "random_tf"]
