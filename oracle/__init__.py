"""FP64 CPU oracle (test infrastructure only; see kriging.py)."""
from .kriging import *  # noqa: F401,F403
from .kriging import (covariance, correlation, semivariogram, covariance_derivatives, edge_path,
                      candidates, floor_order, select_neighbours, bordered_solve, krige_points,
                      krige_volume, krige_sample, loso_loss, loso_loss_grad, loso_fd_grad, adam_fit,
                      window_condition)
