"""The stencil selection that allocates nothing (rbf_select_stencils_static,
for callers that cannot allocate) against the workspace form
(rbf_select_stencils): bit-identical stencils on two calls in a row, the
second on a smaller input, and the size limit of its fixed array."""
import ctypes

import numpy as np
import pytest
import torch

import nodesets as ns
import paper_1912_13282_amd as rb
from paper_1912_13282_amd import _binding as B

pytestmark = pytest.mark.gpu


def _inputs(nd, n, dev):
    off = ns.offsets_from_sizes(np.full(nd.N, n, dtype=np.int64))
    return (torch.from_numpy(nd.X).to(dev), torch.from_numpy(off).to(dev))


def test_static_selection_matches_workspace_form(gpu):
    # first call: the 3D cube minus sphere at full size (1,096,553 nodes, n = 35);
    # second call: the 2,007-node disk with n = 15, on the same array
    cases = [(ns.workload("cube_sphere3d")["nodes"][0], 35), (ns.disk(0.0404, 1001), 15)]
    for nd, n in cases:
        print(f"[no-alloc] N={nd.N} d={nd.X.shape[1]} n={n}", flush=True)
        X, off = _inputs(nd, n, gpu)
        ref = rb.select_stencils(X, off, n)
        torch.cuda.synchronize()
        idx = torch.full_like(ref, -7)
        rb.select_stencils_static(X, off, n, idx=idx)
        torch.cuda.synchronize()
        assert torch.equal(idx, ref)
        assert int(idx[0].item()) == 0


def test_static_selection_ragged_and_repeat(gpu):
    # ragged stencil sizes (1..40) on a torus, called twice on the same array
    nd = ns.torus(0.03, 3)
    rng = np.random.default_rng(9)
    sizes = rng.integers(1, 41, nd.N)
    off = torch.from_numpy(ns.offsets_from_sizes(sizes)).to(gpu)
    X = torch.from_numpy(nd.X).to(gpu)
    ref = rb.select_stencils(X, off, 40)
    for _ in range(2):
        idx = rb.select_stencils_static(X, off, 40)
        torch.cuda.synchronize()
        assert torch.equal(idx, ref)


def test_static_selection_size_limit(gpu):
    # the workspace of 1.7M nodes in 3D exceeds the fixed array: a clear error, nothing launched
    N = 1_700_000
    b = B.select_stencils_workspace(N, 3, 35)
    assert b > B.SELECT_STATIC_BYTES
    X = torch.zeros((N, 3), dtype=torch.float64, device=gpu)
    off = torch.arange(0, (N + 1) * 35, 35, dtype=torch.int64, device=gpu)
    idx = torch.empty(1, dtype=torch.int32, device=gpu)
    ctx = rb.context(gpu)
    st = rb.lib().rbf_select_stencils_static(ctx._sync_stream(), ctypes.c_void_p(X.data_ptr()), N, 3,
                                             ctypes.c_void_p(off.data_ptr()), 35, ctypes.c_void_p(idx.data_ptr()))
    assert st == -4   # RBF_EWORKSPACE
