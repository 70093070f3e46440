"""MI355X-native batched fitting of exponential-kernel multi-dimensional
Hawkes processes (the estimation path of "MDHP-Net", Sec. IV-B).

The computation lives in ``libmdhp.so`` (hand-written HIP for gfx950, C ABI
in ``include/mdhp.h``); this package only marshals arguments.
"""

from .api import (BETA_PAIR, BETA_SHARED, FIT_CONVERGED, FIT_MAX_STEPS, FIT_NONFINITE,
                  FIT_STALLED, OPT_EM, OPT_LBFGS, OPT_PADAM, OPT_PGD, SCATTER_MFMA, FitOptions,
                  MdhpError, Plan,
                  mdhp_check_params, mdhp_cold_start, mdhp_fit_batch, mdhp_grad, mdhp_grad_static,
                  mdhp_simulate, mdhp_attack_times,
                  mdhp_loglik,
                  mdhp_plan_create, mdhp_plan_destroy, mdhp_status_string)
from .autograd import MDHPLogLik, mdhp_loglik_autograd
from .lstm import (MDHPLSTM, MDHPLSTMFunction, mdhp_lstm_backward, mdhp_lstm_forward,
                   mdhp_lstm_phase_ms, mdhp_lstm_sizes, mdhp_lstm_timing)

__all__ = ["Plan", "FitOptions", "MDHPLogLik", "mdhp_loglik_autograd", "MdhpError", "mdhp_plan_create", "mdhp_plan_destroy",
           "mdhp_loglik", "mdhp_grad", "mdhp_grad_static", "mdhp_simulate", "mdhp_attack_times", "mdhp_fit_batch", "mdhp_check_params", "mdhp_cold_start",
           "mdhp_status_string", "BETA_SHARED", "BETA_PAIR", "OPT_PGD", "OPT_PADAM",
           "OPT_LBFGS", "OPT_EM", "SCATTER_MFMA", "FIT_CONVERGED", "FIT_MAX_STEPS", "FIT_NONFINITE", "FIT_STALLED",
           "MDHPLSTM", "MDHPLSTMFunction", "mdhp_lstm_forward", "mdhp_lstm_backward",
           "mdhp_lstm_sizes", "mdhp_lstm_timing", "mdhp_lstm_phase_ms"]
