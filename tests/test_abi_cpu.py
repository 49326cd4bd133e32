"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the GPU.  No
compute call is made here."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_1609_01479_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("liblbmi.so is not built (run __graft_entry__.build())")
    return _abi


def test_header_declares_the_binding_surface(abi):
    assert _declared_functions() == sorted(abi.EXPORTS)


def test_library_exports_every_declared_symbol(abi):
    L = abi.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert L.lb_abi_version() == abi.ABI_VERSION == 5


def _params(abi, **kw):
    base = dict(nx=8, ny=8, nz=8, A=-0.00625, B=0.00625, kappa=0.004, gamma=0.5, tau_f=1.0,
                tau_g=1.0, rho0=1.0, precision=abi.LB_FP64, kernel=0, segment_x=0)
    base.update(kw)
    return abi.LbParams(**base)


def _query(abi, **kw):
    s = abi.LbSizes()
    return abi.lib().lb_query_sizes(ctypes.byref(_params(abi, **kw)), ctypes.byref(s)), s


def test_query_sizes(abi):
    st, s = _query(abi, nx=16, ny=16, nz=16)
    assert st == abi.LB_OK
    assert s.elem_bytes == 8 and s.stride_elems >= 4096 and s.stride_elems % 256 == 0
    assert s.state_bytes == 2 * 19 * s.stride_elems * 8
    st, s32 = _query(abi, nx=16, ny=16, nz=16, precision=abi.LB_FP32_DEV)
    assert st == abi.LB_OK and s32.elem_bytes == 4
    # FP32: f and g in FP32 plus the 32-bit words of the reference order parameter
    assert s32.state_bytes == 2 * 19 * s32.stride_elems * 4 + s32.stride_elems * 4
    assert s32.phi_bytes == s32.stride_elems * 8


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), "LB_ESHAPE"), (dict(ny=-3), "LB_ESHAPE"),
    (dict(nx=2048, ny=2048, nz=1024), "LB_ESHAPE"),
    (dict(nx=1, ny=8192, nz=4096), "LB_ESHAPE"),  # one FP64 x-plane of f >= 4 GiB
    (dict(tau_f=0.5), "LB_EINVAL"), (dict(tau_g=0.2), "LB_EINVAL"),
    (dict(tau_f=float("nan")), "LB_EINVAL"), (dict(rho0=0.0), "LB_EINVAL"),
    (dict(precision=7), "LB_EINVAL"), (dict(kernel=3), "LB_EINVAL"),
    (dict(kernel=-1), "LB_EINVAL"),
    (dict(kernel=2, coupling=1), "LB_EINVAL"), (dict(kernel=2, order_param=1), "LB_EINVAL"),
    (dict(layout=4), "LB_EINVAL"), (dict(layout=-1), "LB_EINVAL"),
    (dict(layout=3, aosoa_len=3), "LB_ESHAPE"), (dict(layout=3, aosoa_len=0), "LB_ESHAPE"),
    (dict(layout=3, aosoa_len=64, nz=96), "LB_ESHAPE"),
    (dict(coupling=2), "LB_EINVAL"), (dict(coupling=-1), "LB_EINVAL"),
    (dict(order_param=2), "LB_EINVAL"), (dict(order_param=-1), "LB_EINVAL"),
])
def test_bad_parameters_rejected(abi, kw, code):
    st, _ = _query(abi, **kw)
    assert st == getattr(abi, code)
    assert abi.lib().lb_last_error().decode()


def test_force_coupling_sizes(abi):
    """The force coupling needs one FP64 work field (phi; Pi is formed on the
    fly) and, for its adjoint, three more scratch components (dL/dF) than
    the stress coupling's five, in either order-parameter scheme."""
    for op in (0, 1):
        for prec, e in ((0, 8), (1, 4)):
            st, s0 = _query(abi, coupling=0, order_param=op, precision=prec)
            st1, s1 = _query(abi, coupling=1, order_param=op, precision=prec)
            assert st == st1 == abi.LB_OK
            assert s0.adj_scratch_bytes == 5 * s0.stride_elems * e
            assert s1.adj_scratch_bytes == 8 * s1.stride_elems * e
            assert s1.phi_bytes == (s1.stride_elems * 8 if op == 0 else 4 * s1.stride_elems * 8)


@pytest.mark.parametrize("prec,e", [(0, 8), (1, 4)])
def test_fd_order_parameter_sizes_and_calls_without_launching(abi, prec, e):
    """The finite-difference order parameter: a level is f then the FP64 phi
    field, 4 FP64 work fields (mu, u), partials for one block per 256 sites;
    g-taking calls reject a g pointer, all before any HIP call."""
    n = 40 * 40 * 40
    st, s = _query(abi, nx=40, ny=40, nz=40, order_param=1, precision=prec)
    assert st == abi.LB_OK
    assert s.state_bytes == 19 * s.stride_elems * e + s.stride_elems * 8
    assert s.phi_bytes == 4 * s.stride_elems * 8
    assert s.scratch_bytes >= 5 * 8 * ((n + 255) // 256)
    L = abi.lib()
    p = _params(abi, order_param=1, precision=prec)
    ctx = ctypes.c_void_p()
    b = abi.LbBuffers()
    b.state[0], b.state[1], b.phi, b.scratch = 0x1000, 0x2000, 0x3000, 0x4000
    b.adj[0], b.adj[1], b.adj_scratch = 0x5000, 0x6000, 0x7000
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
    v = ctypes.c_void_p(0x8000)
    assert L.lb_export_dist(ctx, v, v) == abi.LB_EINVAL
    assert L.lb_import_dist(ctx, v, v) == abi.LB_EINVAL
    assert L.lb_import_dist(ctx, None, None) == abi.LB_EINVAL
    # no g: the adjoint export takes dL/df only
    assert L.lb_adjoint_export(ctx, v, v) == abi.LB_EINVAL
    L.lb_destroy(ctx)


def test_fp32_plane_limit_is_twice_fp64(abi):
    """The per-plane limit counts bytes: the plane that FP64 rejects fits in
    FP32 storage."""
    st, _ = _query(abi, nx=1, ny=8192, nz=4096, precision=abi.LB_FP32_DEV)
    assert st == abi.LB_OK


def test_create_validates_buffers_without_launching(abi):
    """Argument errors return before any HIP call: NULL and misaligned buffers."""
    L = abi.lib()
    p = _params(abi)
    ctx = ctypes.c_void_p()
    b = abi.LbBuffers()
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_EINVAL
    b.state[0], b.state[1], b.phi, b.scratch = 0x1000, 0x2000, 0x3000, 0x4008
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_EALIGN
    b.scratch = 0x4000
    b.adj[0] = 0x5000
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_EINVAL
    b.adj[0] = 0
    b.state[1] = b.state[0]
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_EINVAL
    # a valid set of (fake, never dereferenced) pointers creates a host context
    b.state[1] = 0x2000
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
    assert ctx.value
    assert L.lb_step(ctx, -1) == abi.LB_EINVAL
    assert L.lb_step_from(ctx, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1000)) == abi.LB_EINVAL
    assert L.lb_step_from(ctx, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2010)) == abi.LB_EALIGN
    assert L.lb_step_from(ctx, None, ctypes.c_void_p(0x2000)) == abi.LB_EINVAL
    assert L.lb_adjoint_seed(ctx, ctypes.c_void_p(0x1000)) == abi.LB_ESTATE
    assert L.lb_adjoint_export(ctx, ctypes.c_void_p(0x1000), None) == abi.LB_ESTATE
    assert L.lb_adjoint_export(None, ctypes.c_void_p(0x1000), None) == abi.LB_EINVAL
    L.lb_destroy(ctx)
    b.adj[0], b.adj[1], b.adj_scratch = 0x5000, 0x6000, 0x7000
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
    assert L.lb_adjoint_export(ctx, ctypes.c_void_p(0x1010), None) == abi.LB_EALIGN
    assert L.lb_adjoint_export(ctx, None, ctypes.c_void_p(0x1010)) == abi.LB_EALIGN
    assert L.lb_adjoint_export(ctx, None, None) == abi.LB_OK  # nothing to copy
    L.lb_destroy(ctx)
    L.lb_destroy(None)


def test_step_sums_noalloc_validates_without_launching(abi):
    """lb_step_sums_noalloc rejects a NULL context or output, a negative step
    count and a lattice whose steps reduce over more partial blocks than the
    library's array holds, before any HIP call."""
    L = abi.lib()
    ctx = ctypes.c_void_p()
    b = abi.LbBuffers()
    b.state[0], b.state[1], b.phi, b.scratch = 0x1000, 0x2000, 0x3000, 0x4000
    out = ctypes.c_void_p(0x8000)
    assert L.lb_step_sums_noalloc(None, 1, out) == abi.LB_EINVAL
    # 479^3, the largest cube the kernels accept, fits the array
    for shape, fits in (((479, 479, 479), True), ((1, 100000, 1), False),
                        ((16, 16, 16), True)):
        nx, ny, nz = shape
        st, s = _query(abi, nx=nx, ny=ny, nz=nz)
        assert st == abi.LB_OK
        assert (s.scratch_bytes // 40 <= abi.NOALLOC_MAX_PARTIALS) == fits, shape
        p = _params(abi, nx=nx, ny=ny, nz=nz)
        assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
        assert L.lb_step_sums_noalloc(ctx, 1, None) == abi.LB_EINVAL
        assert L.lb_step_sums_noalloc(ctx, -1, out) == abi.LB_EINVAL
        if not fits:
            assert L.lb_step_sums_noalloc(ctx, 1, out) == abi.LB_EINVAL
            assert b"partial blocks" in L.lb_last_error()
        L.lb_destroy(ctx)


@pytest.mark.parametrize("prec", [0, 1])
def test_phi_taking_calls_validate_without_launching(abi, prec):
    """lb_step_from_phi and lb_adjoint_step_phi (either storage) reject a
    missing context, phi field or adjoint, misaligned pointers, equal levels
    and the finite-difference scheme before any HIP call."""
    L = abi.lib()
    a1, a2, bad = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2010)
    phi = ctypes.c_void_p(0x3000)
    for fd in (0, 1):
        p = _params(abi, precision=prec, order_param=fd)
        ctx = ctypes.c_void_p()
        b = abi.LbBuffers()
        b.state[0], b.state[1], b.phi, b.scratch = 0x1000, 0x2000, 0x3000, 0x4000
        assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
        if fd:
            assert L.lb_step_from_phi(ctx, a1, a2, phi) == abi.LB_EINVAL
            assert L.lb_adjoint_step_phi(ctx, a1, phi, None) == abi.LB_EINVAL
            L.lb_destroy(ctx)
            continue
        assert L.lb_adjoint_step_phi(ctx, a1, phi, None) == abi.LB_ESTATE  # no adjoint buffers
        assert L.lb_step_from_phi(None, a1, a2, phi) == abi.LB_EINVAL
        assert L.lb_step_from_phi(ctx, a1, a2, None) == abi.LB_EINVAL
        assert L.lb_step_from_phi(ctx, a1, a2, bad) == abi.LB_EALIGN
        assert L.lb_step_from_phi(ctx, a1, a1, phi) == abi.LB_EINVAL
        assert L.lb_step_from_phi(ctx, a1, bad, phi) == abi.LB_EALIGN
        L.lb_destroy(ctx)
        b.adj[0], b.adj[1], b.adj_scratch = 0x5000, 0x6000, 0x7000
        assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
        assert L.lb_adjoint_step_phi(None, a1, phi, None) == abi.LB_EINVAL
        assert L.lb_adjoint_step_phi(ctx, a1, None, None) == abi.LB_EINVAL
        assert L.lb_adjoint_step_phi(ctx, None, phi, None) == abi.LB_EINVAL
        assert L.lb_adjoint_step_phi(ctx, a1, bad, None) == abi.LB_EALIGN
        assert L.lb_adjoint_step_phi(ctx, bad, phi, None) == abi.LB_EALIGN
        L.lb_destroy(ctx)


def test_struct_layouts_and_enums_match_the_header(abi, tmp_path):
    """The ctypes structures and constants of the binding agree with
    include/lb.h as a C compiler lays them out (sizeof, every field's
    offset, every enum value the binding and lb.py use)."""
    import subprocess

    from paper_1609_01479_amd import lb as lbpy
    structs = {"lb_params": abi.LbParams, "lb_sizes": abi.LbSizes, "lb_buffers": abi.LbBuffers}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lb.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    enums = {"LB_OK": abi.LB_OK, "LB_EINVAL": abi.LB_EINVAL, "LB_ESHAPE": abi.LB_ESHAPE,
             "LB_EALIGN": abi.LB_EALIGN, "LB_EHIP": abi.LB_EHIP, "LB_ESTATE": abi.LB_ESTATE,
             "LB_FP64": abi.LB_FP64, "LB_FP32_DEV": abi.LB_FP32_DEV,
             "LB_KERNEL_FUSED": abi.LB_KERNEL_FUSED, "LB_KERNEL_TWO_PASS": abi.LB_KERNEL_TWO_PASS,
             "LB_KERNEL_STREAM": abi.LB_KERNEL_STREAM,
             "LB_NVEL": abi.NVEL, "LB_ABI_VERSION": abi.lib().lb_abi_version(),
             "LB_LAYOUT_ROWS": lbpy.LAYOUTS["rows"], "LB_LAYOUT_SOA": lbpy.LAYOUTS["soa"],
             "LB_LAYOUT_AOS": lbpy.LAYOUTS["aos"], "LB_LAYOUT_AOSOA": lbpy.LAYOUTS["aosoa"],
             "LB_COUPLING_STRESS": lbpy.COUPLINGS["stress"],
             "LB_COUPLING_FORCE": lbpy.COUPLINGS["force"],
             "LB_OP_LB": lbpy.ORDER_PARAMS["lb"], "LB_OP_FD": lbpy.ORDER_PARAMS["fd"],
             "LB_NOALLOC_MAX_PARTIALS": abi.NOALLOC_MAX_PARTIALS}
    for name in enums:
        lines.append(f'printf("enum {name} %d\\n", (int){name});')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    for name, val in enums.items():
        assert got[("enum", name)] == val, name


def test_status_strings(abi):
    L = abi.lib()
    for code in range(6):
        assert L.lb_status_string(code)


def test_shard_sizes_and_validation(abi):
    """An x-slab shard (halo_x): levels hold two halo planes on each side, a
    face buffer is 24 component planes (+ the plane of phi_c words in FP32
    storage); shards reject what they do not support, before any HIP call."""
    for prec, e in ((0, 8), (1, 4)):
        st, s = _query(abi, nx=6, ny=10, nz=12, precision=prec, halo_x=1)
        assert st == abi.LB_OK
        assert s.stride_elems >= (6 + 4) * 10 * 12
        a = 10 * 12
        assert s.face_bytes == (24 * a * e + (a * 4 if e == 4 else 0) + 255) // 256 * 256
        st, s0 = _query(abi, nx=6, ny=10, nz=12, precision=prec)
        assert st == abi.LB_OK and s0.face_bytes == 0
    for kw, code in ((dict(nx=1), "LB_ESHAPE"), (dict(coupling=1), "LB_EINVAL"),
                     (dict(order_param=1), "LB_EINVAL"), (dict(kernel=1), "LB_EINVAL"),
                     (dict(halo_x=2), "LB_EINVAL")):
        base = dict(halo_x=1)
        base.update(kw)
        st, _ = _query(abi, **base)
        assert st == getattr(abi, code), kw
    st, _ = _query(abi, halo_x=1, kernel=2)
    assert st == abi.LB_OK
    L = abi.lib()
    ctx = ctypes.c_void_p()
    b = abi.LbBuffers()
    b.state[0], b.state[1], b.phi, b.scratch = 0x1000, 0x2000, 0x3000, 0x4000
    b.adj[0], b.adj[1], b.adj_scratch = 0x5000, 0x6000, 0x7000
    p = _params(abi, halo_x=1)
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
    v, w = ctypes.c_void_p(0x8000), ctypes.c_void_p(0x9000)
    assert L.lb_step(ctx, 2) == abi.LB_EINVAL
    assert L.lb_import_dist(ctx, v, w) == abi.LB_ESTATE
    assert L.lb_adjoint_seed(ctx, v) == abi.LB_ESTATE
    assert L.lb_adjoint_step(ctx, v, None) == abi.LB_ESTATE
    assert L.lb_pack_faces(ctx, ctypes.c_void_p(0x8010), None) == abi.LB_EALIGN
    assert L.lb_unpack_faces(ctx, v, v) == abi.LB_EINVAL
    assert L.lb_pack_faces(ctx, None, None) == abi.LB_OK
    L.lb_destroy(ctx)
    p = _params(abi)
    assert L.lb_create(ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(ctx)) == abi.LB_OK
    assert L.lb_pack_faces(ctx, v, w) == abi.LB_ESTATE
    assert L.lb_unpack_faces(ctx, v, w) == abi.LB_ESTATE
    L.lb_destroy(ctx)
