"""Acoustic wave-equation forward operator and adjoint-state gradient on AMD MI355X (gfx950).

The computation lives in libawe.so (hand-written HIP kernels behind a C ABI, include/awe.h);
this package is its Python binding and a torch.autograd rule.  Nothing here computes the
operators itself, and nothing falls back to the CPU.
"""
from .binding import (AWE_ERR_CFL, AWE_ERR_NONFINITE, AWE_ERR_WORKSPACE, CHECK_INPUTS, CHECK_LAUNCHES, CHECK_OUTPUTS, EXPORTS,
                      FUSE_ADJOINT, FUSE_BOTH, FUSE_FORWARD, FUSE_NONE, LIB_PATH, PREC_BF16, PREC_FP16, PREC_FP32,
                      STORE_AUTO, STORE_CHECKPOINT, STORE_FULL, STORE_NONE, STORE_PROBED, AweError, Plan, ShotGeometry, Storage,
                      checkpoint_schedule, dot, lib, patchy, patchy_vjp, residual, residual_noalloc,
                      select_storage, slowness2, velocity_gradient)

__all__ = ["AWE_ERR_CFL", "AWE_ERR_NONFINITE", "AWE_ERR_WORKSPACE", "CHECK_INPUTS", "CHECK_LAUNCHES", "CHECK_OUTPUTS", "EXPORTS",
           "FUSE_ADJOINT", "FUSE_BOTH", "FUSE_FORWARD", "FUSE_NONE", "LIB_PATH", "PREC_BF16", "PREC_FP16", "PREC_FP32",
           "STORE_AUTO", "STORE_CHECKPOINT", "STORE_FULL", "STORE_NONE", "STORE_PROBED", "AweError", "Plan", "ShotGeometry", "Storage",
           "checkpoint_schedule", "dot", "lib", "patchy", "patchy_vjp", "residual", "residual_noalloc",
           "select_storage", "slowness2",
           "velocity_gradient", "WaveOp", "wave_forward", "extend_edge", "misfit", "Slowness2",
           "slowness2_from_velocity", "Patchy", "patchy_rock_physics", "BornOp", "born_forward"]


def __getattr__(name):
    if name in ("WaveOp", "wave_forward", "extend_edge", "misfit", "Slowness2", "slowness2_from_velocity",
                "Patchy", "patchy_rock_physics", "BornOp", "born_forward"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
