"""FP64 CPU oracle for the SR-MRA EM step -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package.  The product path (paper_2204_04754_amd) never imports
it and shares no code with it.
"""
from .em_oracle import (  # noqa: F401
    forward, shift_downsample_indices, log_joint, logsumexp_over_shifts,
    log_likelihood, posterior, m_step_sums, em_sums, merge_sums, em_finish, em_step, q_function,
    dense_operators, dense_x_step, hard_assignment_posterior,
)
