"""FP64 CPU oracle for DNA KL-NMF (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP path.
"""
from .dna_oracle import (ALPHA, EPS, DomainError, FitResult, StepResult,  # noqa: F401
                         fit_dna, fit_mu, h_step, kl_cost, kl_divergence,
                         mu_h_step, mu_w_step, newton_candidate, normalize,
                         normalize_h_rows, normalize_w_columns, objective, partial_cost,
                         ratios, renormalize, unrolled_h, w_step)
