"""FP64 CPU oracle (test infrastructure only; see ttt_oracle's header)."""
from .ttt_oracle import (  # noqa: F401
    NORM_EPS, activation, l2norm_rows, l2norm_rows_bwd, chunk_bounds, fast_forward,
    inner_loss, inner_grad, ttt_forward, ttt_forward_batched, ttt_backward, ttt_backward_batched, outer_objective,
    ttt_forward_gcs, ttt_backward_gcs, swiglu_forward, swiglu_dot_loss, swiglu_dot_grad, ttt_forward_swiglu,
    swiglu_apply_adjoint, swiglu_update_adjoint, ttt_backward_swiglu, gcm_layer_forward, gcm_layer_backward,
)
