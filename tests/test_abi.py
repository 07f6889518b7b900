"""The C-ABI library builds for gfx950, loads, and exports every symbol the header declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_1912_13282_amd", "librbffd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_1912_13282_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for n in ["rbf_select_stencils", "rbf_compute_weights", "rbf_assemble_csr", "rbf_ctx_create"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s+(rbf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_with_ctypes(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    for n in declared():
        assert hasattr(L, n)
    L.rbf_status_string.restype = ctypes.c_char_p
    assert L.rbf_status_string(-4) == b"workspace too small"


def test_host_argument_errors_without_gpu(lib_path):
    """Argument checks run on the host before any device call."""
    import ctypes
    L = ctypes.CDLL(lib_path)
    b = ctypes.c_size_t()
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 4, 10, ctypes.byref(b)) == -3   # EDIM
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 3, 10, None) == -1              # EINVAL
    assert L.rbf_select_stencils_workspace(ctypes.c_int64(1000), 3, 10, ctypes.byref(b)) == 0
    assert b.value > 1000 * (4 + 8 * 3)
    assert L.rbf_compute_weights(None, None, ctypes.c_int64(0), 2, None, None, ctypes.c_int64(0), 1, None, 2, 1,
                                 None, None, None) == -1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's sizes and offsets."""
    import ctypes
    from paper_1912_13282_amd import _binding as B
    src = tmp_path / "lay.c"
    src.write_text(f'''#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
#define F(T, f) printf(#T " " #f " %zu\\n", offsetof(T, f));
int main(void) {{
  printf("rbf_options size %zu\\n", sizeof(rbf_options));
  F(rbf_options, precision) F(rbf_options, max_refine) F(rbf_options, phs_power) F(rbf_options, scale_mode)
  F(rbf_options, repro_tol) F(rbf_options, refine_tol) F(rbf_options, surrogate_tol)
  F(rbf_options, surrogate_corr_tol)
  printf("rbf_domain_desc size %zu\\n", sizeof(rbf_domain_desc));
  F(rbf_domain_desc, X) F(rbf_domain_desc, N) F(rbf_domain_desc, d) F(rbf_domain_desc, offsets)
  F(rbf_domain_desc, idx) F(rbf_domain_desc, nnz) F(rbf_domain_desc, degree) F(rbf_domain_desc, degree_uniform)
  F(rbf_domain_desc, n_max) F(rbf_domain_desc, op_mask) F(rbf_domain_desc, w) F(rbf_domain_desc, status)
  printf("rbf_plan size %zu\\n", sizeof(rbf_plan));
  F(rbf_plan, chunk) F(rbf_plan, waves_per_cu) F(rbf_plan, ms)
  printf("rbf_solve_info size %zu\\n", sizeof(rbf_solve_info));
  F(rbf_solve_info, status) F(rbf_solve_info, iterations) F(rbf_solve_info, residual) F(rbf_solve_info, true_residual)
  return 0;
}}
''')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-O0", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    py = {"rbf_options": B.rbf_options, "rbf_domain_desc": B.rbf_domain_desc, "rbf_plan": B.rbf_plan,
          "rbf_solve_info": B.rbf_solve_info}
    for line in filter(None, out):
        T, f, v = line.split()
        if f == "size":
            assert ctypes.sizeof(py[T]) == int(v), T
        else:
            assert getattr(py[T], f).offset == int(v), (T, f)


def test_mlp_parameter_layout():
    """Flat parameter order W1, b1, ..., W4, b4 with the header's count."""
    import torch
    from paper_1912_13282_amd import _binding as B
    src = open(HEADER).read()
    assert int(re.search(r"#define RBF_MLP_NPARAM\s+(\d+)", src).group(1)) == B.MLP_NPARAM
    shapes = dict(B.MLP_SHAPES)
    assert sum(int(torch.tensor(s).prod()) for s in shapes.values()) == B.MLP_NPARAM
    p = {k: torch.full(s, float(i)) for i, (k, s) in enumerate(B.MLP_SHAPES)}
    flat = B.mlp_flatten(p)
    back = B.mlp_unflatten(flat)
    for k in p:
        assert torch.equal(back[k], p[k])
    assert flat[0] == 0 and flat[128 * 30] == 1 and flat[-1] == 7


def test_defaults_and_status_strings(lib_path):
    import ctypes
    from paper_1912_13282_amd import _binding as B
    L = ctypes.CDLL(lib_path)
    o = B.rbf_options()
    assert L.rbf_options_default(ctypes.byref(o)) == 0
    assert (o.precision, o.max_refine, o.phs_power, o.scale_mode) == (0, 10, 3, 0)
    assert (o.repro_tol, o.refine_tol, o.surrogate_tol, o.surrogate_corr_tol) == (1e-8, 0.0, 1e-6, 0.25)
    L.rbf_status_string.restype = ctypes.c_char_p
    texts = {c: L.rbf_status_string(c) for c in (0, -1, -2, -3, -4, -5, -6, -7)}
    assert len(set(texts.values())) == 8 and texts[-7] == b"unknown status"


def test_more_host_argument_errors_without_gpu(lib_path):
    """Every entry point rejects a missing context or inconsistent sizes on the host."""
    import ctypes
    from paper_1912_13282_amd import _binding as B
    L = ctypes.CDLL(lib_path)
    b = ctypes.c_size_t()
    # batched: domain count outside [1, 16], missing arrays
    D = (B.rbf_domain_desc * 17)()
    assert L.rbf_batched_workspace(D, 0, ctypes.byref(b)) == -1
    assert L.rbf_batched_workspace(D, 17, ctypes.byref(b)) == -1
    assert L.rbf_batched_workspace(D, 1, ctypes.byref(b)) == -1          # X, offsets... are NULL
    D[0].X = D[0].offsets = D[0].idx = D[0].w = D[0].status = ctypes.c_void_p(16)
    D[0].N, D[0].nnz, D[0].n_max, D[0].d, D[0].op_mask, D[0].degree_uniform = 100, 1500, 15, 4, 1, 2
    assert L.rbf_batched_workspace(D, 1, ctypes.byref(b)) == -3          # EDIM
    D[0].d = 2
    D[0].degree_uniform = 5
    assert L.rbf_batched_workspace(D, 1, ctypes.byref(b)) == -6          # degree beyond 4
    D[0].degree_uniform = 2
    D[0].n_max = 101
    assert L.rbf_batched_workspace(D, 1, ctypes.byref(b)) == -2          # ETOOFEW
    D[0].n_max = 15
    assert L.rbf_batched_workspace(D, 1, ctypes.byref(b)) == 0 and b.value >= 100 * 16
    assert L.rbf_compute_weights_batched(None, D, 1, None, None, ctypes.c_size_t(0)) == -1
    # surrogate and MLP entry points
    assert L.rbf_mlp_grad_workspace(ctypes.c_int64(0), ctypes.byref(b)) == -1
    assert L.rbf_mlp_grad_workspace(ctypes.c_int64(130), ctypes.byref(b)) == 0 and b.value == 3 * 38976 * 4
    assert L.rbf_mlp_pack(None, None, None) == -1
    assert L.rbf_surrogate_load(None, None) == -1
    assert L.rbf_assemble_csr(None, ctypes.c_int64(1), None, None, None, 0, ctypes.c_int64(1), 1, None, None,
                              None) == -1
    # explicit evaluation, implicit assembly and the solver
    one = ctypes.c_int64(1)
    assert L.rbf_apply_operators(None, one, None, None, None, 1, one, 1, None, one, None) == -1
    assert L.rbf_explicit_step(None, one, 2, None, None, one, 1, None, None, None, None, None, None, None,
                               ctypes.c_double(0.1), None) == -1
    assert L.rbf_assemble_implicit(None, one, 2, None, None, one, None, None, None, None, None, None, None,
                                   None) == -1
    I64 = ctypes.c_int64
    assert L.rbf_bicgstab_workspace(I64(0), I64(0), 1, ctypes.byref(b)) == -1
    assert L.rbf_bicgstab_workspace(I64(1000), I64(9000), 1, None) == -1
    assert L.rbf_bicgstab_workspace(I64(1000), I64(-1), 1, ctypes.byref(b)) == -1
    assert L.rbf_bicgstab_workspace(I64(1000), I64(9000), 7, ctypes.byref(b)) == -1
    assert L.rbf_bicgstab_workspace(I64(1000), I64(9000), 1, ctypes.byref(b)) == 0
    assert b.value >= 9 * 1000 * 8 + 5120 * 8
    jac = b.value
    assert L.rbf_bicgstab_workspace(I64(1000), I64(9000), 2, ctypes.byref(b)) == 0
    assert b.value >= jac + 12 * (9000 + 1000) + 24 * 1000
    assert L.rbf_bicgstab(None, one, None, None, None, one, 1, None, None, ctypes.c_double(1e-8), 10, 1, None,
                          ctypes.c_size_t(0), None, ctypes.c_size_t(0), None) == -1
    assert L.rbf_block_jacobi_size(ctypes.c_int64(1000), 4, ctypes.byref(b)) == -3
    assert L.rbf_block_jacobi_size(ctypes.c_int64(1000), 3, ctypes.byref(b)) == 0
    assert b.value >= 1000 * (8 + 128 + 4)  # node order and its inverse, float16 rows and their scales


def test_node_kind_and_solver_constants_match_the_binding():
    from paper_1912_13282_amd import _binding as B
    src = open(HEADER).read()
    val = lambda name: int(re.search(r"#define " + name + r"\s+(\d+)", src).group(1))  # noqa: E731
    assert (val("RBF_NODE_INTERIOR"), val("RBF_NODE_DIRICHLET"), val("RBF_NODE_NEUMANN")) == \
        (B.NODE_INTERIOR, B.NODE_DIRICHLET, B.NODE_NEUMANN)
    assert (val("RBF_SOLVE_CONVERGED"), val("RBF_SOLVE_MAXITER"), val("RBF_SOLVE_BREAKDOWN"),
            val("RBF_SOLVE_BADDIAG"), val("RBF_SOLVE_DIVERGED")) == \
        (B.SOLVE_CONVERGED, B.SOLVE_MAXITER, B.SOLVE_BREAKDOWN, B.SOLVE_BADDIAG, B.SOLVE_DIVERGED)
    assert (val("RBF_PRECOND_NONE"), val("RBF_PRECOND_JACOBI"), val("RBF_PRECOND_BLOCK_JACOBI")) == \
        (B.PRECOND["none"], B.PRECOND["jacobi"], B.PRECOND["block_jacobi"])
