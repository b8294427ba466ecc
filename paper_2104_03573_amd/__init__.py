"""MI355X-native deviational phonon Monte Carlo tracer (HIP kernels behind a C ABI).

The public Python surface mirrors include/mcbte.h: build_tables, free_tables, table_info,
table_export, state_bytes, emit, trace, batch_queue_bytes, trace_batch, trace_batch_static, adjoint,
adjoint_finalize, tally, tally_batches, kappa_cumulative, strerror.
"""
from .mcbte import (COUNT_NAMES, ESTIMATORS, EXPORTED, LIB_PATH, SENS_LOCAL, SENS_PATHWISE, SENS_SCORE, MCBTEError, Tables,
                    adjoint, adjoint_finalize,
                    batch_queue_bytes, build_tables, emit, free_tables, lib, make_run, run, sensitivities,
                    state_bytes, strerror, table_export, table_info, tally, trace, trace_batch, trace_batch_static,
                    tally_batches, kappa_cumulative)

__all__ = ["COUNT_NAMES", "ESTIMATORS", "EXPORTED", "LIB_PATH", "SENS_LOCAL", "SENS_PATHWISE", "SENS_SCORE", "MCBTEError", "Tables",
           "adjoint", "adjoint_finalize",
           "batch_queue_bytes", "build_tables", "emit", "free_tables", "lib", "make_run", "run", "sensitivities",
           "state_bytes", "strerror", "table_export", "table_info", "tally", "trace", "trace_batch",
           "trace_batch_static", "tally_batches", "kappa_cumulative"]

from .mcbte import TUNE_CANDIDATES, autotune, tune, tune_candidate  # noqa: E402
from .autograd import KappaOfTau, kappa_of_tau, tau_bins, with_tau_bins  # noqa: E402

__all__ += ["KappaOfTau", "kappa_of_tau", "tau_bins", "with_tau_bins", "TUNE_CANDIDATES", "autotune", "tune",
            "tune_candidate"]
