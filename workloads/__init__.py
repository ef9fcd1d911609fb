"""Seeded synthetic workloads for the GenEO-PCG solver.

This package only builds *inputs*: tensor-grid node coordinates, per-element
material ids / ply angles / diffusion coefficients, Dirichlet masks, loads and
subdomain cuts.  It contains none of the method's arithmetic (no element
integrals, no decomposition sets, no solves), so that both the CPU oracle and
the GPU library can consume it without sharing any computational code.
"""
from .generate import (Workload, laminate_plate, diffusion_box, spe10_like,
                       config_c1, config_c2, config_c3, config_c5, small_case,
                       PLY_CONSTS, RESIN_CONSTS, iso_consts)

__all__ = ["Workload", "laminate_plate", "diffusion_box", "spe10_like",
           "config_c1", "config_c2", "config_c3", "config_c5", "small_case",
           "PLY_CONSTS", "RESIN_CONSTS", "iso_consts"]
