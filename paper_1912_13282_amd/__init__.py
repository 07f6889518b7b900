"""MI355X-native RBF-FD stencil hot path (Medusa, Slak & Kosec, Sec. 2.1-2.3).

Python face of the HIP library ``librbffd.so`` (C ABI in include/rbffd.h):

    select_stencils  -- exact k-nearest-neighbour stencils, self first
    select_stencils_static
                     -- the same without a workspace (fixed library array), for
                        callers that cannot allocate
    compute_weights  -- RBF-FD weights of the augmented PHS + monomial system
    compute_weights_wls
                     -- GWLS weights (monomial basis, Gaussian or unit weight function)
    assemble_csr     -- the sparse operator in CSR form
    apply_operators  -- explicit evaluation w^T u_{I(i)} of the operators on a field
    combine_operators
                     -- the general second-order operator from stored weights (eq. gen-op)
    explicit_step    -- one explicit Euler step (interior, Dirichlet and Neumann nodes)
    assemble_implicit / bicgstab
                     -- the implicit system M u = r and its BiCGStab solution on the GPU
    compute_weights_batched / autotune_batched
                     -- mixed 2D/3D, per-node degree and size in one persistent launch
    mlp_* / surrogate_*
                     -- the learned 2D Laplacian surrogate: MFMA forward/backward, Adam,
                        projection onto the reproduction conditions, plain-solve fallback

PyTorch supplies device memory and streams only.
"""
from ._binding import (  # noqa: F401
    OPS, ST_BADSIZE, ST_FALLBACK, ST_OK, ST_REFINED, ST_SINGULAR, ST_SURROGATE, ST_SURROGATE_REJECTED,
    Context, Domain, RbfError, assemble_csr, autotune_batched, compute_weights, compute_weights_batched, context,
    batched_class_sizes, get_plan, lib, select_stencils, select_stencils_static, set_plan, compute_weights_wls,
    NODE_DIRICHLET, NODE_INTERIOR, NODE_NEUMANN, apply_operators, combine_operators, explicit_step,
    SOLVE_BADDIAG, SOLVE_BREAKDOWN, SOLVE_CONVERGED, SOLVE_DIVERGED, SOLVE_MAXITER, assemble_implicit, bicgstab,
    bicgstab_workspace, block_jacobi, block_jacobi_size,
    MLP_NPARAM, mlp_adam, mlp_flatten, mlp_forward, mlp_grad, mlp_pack, mlp_unflatten, surrogate_dataset,
    surrogate_load, surrogate_weights,
)
