"""The C-ABI library loads, exports every symbol of include/helmholtz6.h and
include/h6net.h and rejects invalid plans before touching the GPU (no GPU
needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1212_1397_amd", "libhelmholtz6.so")
HEADER = os.path.join(ROOT, "include", "helmholtz6.h")
NET_HEADER = os.path.join(ROOT, "include", "h6net.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(helmholtz6_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("helmholtz6_setup", "helmholtz6_apply_A", "helmholtz6_apply_Pinv", "helmholtz6_solve",
              "helmholtz6_destroy", "helmholtz6_dims", "helmholtz6_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def net_declared_functions():
    text = open(NET_HEADER).read()
    return sorted(set(re.findall(r"\b((?:h6net|helmholtz6)_[a-z_A-Z0-9]+)\s*\(", text)))


def test_binding_lists_every_symbol():
    from paper_1212_1397_amd import helmholtz6 as h6
    assert sorted(h6.EXPORTED) == declared_functions()
    assert sorted(h6.EXPORTED_NET) == net_declared_functions()


def test_library_exports_every_network_symbol():
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB)
    for n in net_declared_functions():
        assert hasattr(lib, n), n


def test_network_parameter_count():
    from paper_1212_1397_amd import helmholtz6 as h6
    from oracle import unet
    assert [(l[0], l[1], l[2]) for l in unet.LAYERS] == list(h6.NET_LAYERS)
    expected = sum(co * ci * 27 + co for _, ci, co in h6.NET_LAYERS)
    assert h6._lib.h6net_param_count() == expected


def test_network_rejects_bad_arguments():
    from paper_1212_1397_amd import helmholtz6 as h6
    out = ctypes.c_void_p()
    bad = (ctypes.c_int * 3)(0, 4, 4)
    assert h6._lib.h6net_create(bad, None, ctypes.byref(out)) == h6.H6_ERR_ARG
    assert not out.value
    big = (ctypes.c_int * 3)(400, 400, 400)      # 48 * 400^3 >= 2^31: beyond 32-bit activation offsets
    assert h6._lib.h6net_create(big, None, ctypes.byref(out)) == h6.H6_ERR_ARG
    assert not out.value
    assert h6._lib.h6net_forward(None, None, 0.0, None, None) == h6.H6_ERR_ARG
    assert h6._lib.helmholtz6_attach_net(None, None) == h6.H6_ERR_ARG
    loss = ctypes.c_double()
    assert h6._lib.h6net_gradients_op(None, None, None, None, None, ctypes.byref(loss), None) == h6.H6_ERR_ARG
    assert h6._lib.h6net_train_step_op(None, None, None, None, 1e-3, ctypes.byref(loss), None) == h6.H6_ERR_ARG


def test_pack_unpack_roundtrip():
    import numpy as np
    from paper_1212_1397_amd import helmholtz6 as h6
    from paper_1212_1397_amd.workloads import init_net_params
    p = init_net_params(h6.NET_LAYERS, 3)
    flat = h6.pack_net_params(p)
    q = h6.unpack_net_params(flat)
    for name, _, _ in h6.NET_LAYERS:
        np.testing.assert_array_equal(q[name][0], p[name][0].astype(np.float32))


def test_status_strings():
    from paper_1212_1397_amd import helmholtz6 as h6
    for st in (0, 1, 2, -1, -2, -3, -4, -5):
        assert h6.status_string(st) and h6.status_string(st) != "unknown status"


@pytest.mark.parametrize("bc,status", [("SSDDDD", -2), ("DDSSDD", -2), ("DNDDDD", -2), ("DDNDDD", -2)])
def test_unsupported_faces_rejected(bc, status):
    from paper_1212_1397_amd import helmholtz6 as h6
    with pytest.raises(h6.H6Error) as e:
        h6.Plan(8, 1 / 9, 3.0, bc)
    assert e.value.status == status


@pytest.mark.parametrize("kw", [dict(n=0, h=0.1), dict(n=4, h=-1.0), dict(n=4, h=float("nan")),
                                dict(n=4, h=0.2, k=float("inf"))])
def test_invalid_arguments_rejected(kw):
    from paper_1212_1397_amd import helmholtz6 as h6
    k = kw.pop("k", 1.0)
    with pytest.raises(h6.H6Error) as e:
        h6.Plan(kw["n"], kw["h"], k)
    assert e.value.status == -1


def test_singular_preconditioner_rejected_at_setup():
    """k^2 h^2 = 12 sin^2(pi h / 2): the (1,1,1) mode of A_p vanishes (host-side check)."""
    import math
    from paper_1212_1397_amd import helmholtz6 as h6
    n = 8
    h = 1.0 / (n + 1)
    k = math.sqrt(12.0 * math.sin(math.pi * h / 2) ** 2) / h
    with pytest.raises(h6.H6Error) as e:
        h6.Plan(n, h, k)
    assert e.value.status == -5


def test_psi_order_matches_definition():
    import math
    from paper_1212_1397_amd import helmholtz6 as h6
    from oracle import psi_order
    assert math.isclose(h6.psi_order(1.0, 0.04, 1.0, 0.16, 2.0), psi_order(0.04, 0.16, 2.0), rel_tol=1e-14)
    assert math.isclose(h6.psi_order(2.0, 0.5, 3.0, 0.75, 2.0), 0.0, abs_tol=1e-15)
    assert math.isnan(h6.psi_order(0.0, 1.0, 1.0, 1.0, 2.0))
    assert math.isnan(h6.psi_order(1.0, 1.0, 1.0, 1.0, 1.0))


def test_rhs_entry_points_reject_bad_arguments():
    """Argument checks happen before any device work: a null plan is refused."""
    from paper_1212_1397_amd import helmholtz6 as h6
    lib = h6._lib
    assert lib.helmholtz6_rhs_separable(None, 1, None, None, None, None, None, None) == h6.H6_ERR_ARG
    assert lib.helmholtz6_rhs_dirichlet_z(None, 0, None, None, None) == h6.H6_ERR_ARG


@pytest.mark.parametrize("n,precision", [((5000, 8, 8), "fp64"), ((8, 5000, 8), "fp64"), ((8, 8, 600), "fp64"),
                                         ((4100, 8, 8), "mixed")])
def test_grids_beyond_kernel_limits_rejected(n, precision):
    """Setup refuses grids beyond the kernels' limits: z lines longer than the
    partitioned solver holds (n'z > 544), x / y lines longer than 4096 (the
    dense transforms' basis matrices); host-side checks, before any device
    allocation."""
    from paper_1212_1397_amd import helmholtz6 as h6
    with pytest.raises(h6.H6Error) as e:
        h6.Plan(n, 1.0 / (max(n) + 1), 2.0, precision=precision)
    assert e.value.status == -1


def test_set_graphs_rejects_unknown_mode():
    from paper_1212_1397_amd import helmholtz6 as h6
    assert h6._lib.helmholtz6_set_graphs(None, 1) == h6.H6_ERR_ARG


def test_rhs_neumann_rejects_bad_arguments():
    from paper_1212_1397_amd import helmholtz6 as h6
    assert h6._lib.helmholtz6_rhs_neumann(None, 4, 1, None, None, None, None, None) == h6.H6_ERR_ARG
