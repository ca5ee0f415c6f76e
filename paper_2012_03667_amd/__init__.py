"""MI355X (gfx950) solver for the vacuum quark gap equation with the Ball-Chiu
vertex (Huang, Duan, Hu, Chen, arXiv:2012.03667).

The compute path is the HIP library ``libqdse.so`` (C ABI in include/qdse.h);
this package only marshals arguments: PyTorch supplies device memory and the
stream. If the library is missing every entry point raises.
"""
from ._lib import (QDSE_AUTO, QDSE_CONV_ABS, QDSE_CONV_MASS, QDSE_EDEVICE, QDSE_EDIVERGED,
                   QDSE_EINVAL, QDSE_ENAN, QDSE_ENOMEM, QDSE_ENOTSUP, QDSE_ESPURIOUS, QDSE_NEWTON,
                   QDSE_PICARD, QDSE_FP32_REFINE, QDSE_FP64, QDSE_FP64_MATRIX,
                   QDSE_NOT_CONVERGED, QDSE_OK, FredSolver, MuSolver, QdseError, Solver,
                   fred_nodes, grid_nodes, library_path, load, measure_launch_floor,
                   measure_peaks, mu_grid_nodes, mu_solve_group, solve_group)

__all__ = ["Solver", "MuSolver", "FredSolver", "fred_nodes", "measure_peaks",
           "measure_launch_floor", "solve_group", "mu_solve_group", "QdseError", "grid_nodes", "mu_grid_nodes",
           "load", "library_path", "QDSE_OK", "QDSE_NOT_CONVERGED", "QDSE_EINVAL", "QDSE_ENOMEM",
           "QDSE_EDEVICE", "QDSE_ENAN", "QDSE_ENOTSUP", "QDSE_EDIVERGED", "QDSE_ESPURIOUS",
           "QDSE_PICARD", "QDSE_NEWTON", "QDSE_AUTO", "QDSE_FP64", "QDSE_FP32_REFINE",
           "QDSE_FP64_MATRIX", "QDSE_CONV_ABS", "QDSE_CONV_MASS"]
