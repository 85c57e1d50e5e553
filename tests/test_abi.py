"""The C ABI: every function declared in include/cast.h is exported by
libcast.so, and argument validation rejects bad input before any device work
(all of these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2503_19894_amd as cast
from circuits import Gate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EINVAL = -1   # cast_status CAST_EINVAL


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cast.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*([A-Za-z_][A-Za-z_0-9]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names) - {"if", "while"})


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15, names
    lib = ctypes.CDLL(cast.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in cast.h but not exported"
        assert n in cast.SIGNATURES, f"{n} has no binding signature"


def test_binding_names_match_header():
    assert set(cast.SIGNATURES) == set(declared_functions())


def _code(fn, *args):
    with pytest.raises(cast.CastError) as ei:
        fn(*args)
    return ei.value.code


def test_sv_create_validation():
    h = ctypes.c_void_p()
    assert _code(cast.sv_create, 0, cast.C128, None, ctypes.byref(h)) == -1
    assert _code(cast.sv_create, 35, cast.C128, None, ctypes.byref(h)) == -1
    assert _code(cast.sv_create, 4, 7, None, ctypes.byref(h)) == -1
    assert "n must be" in cast.last_error() or "dtype" in cast.last_error()


def test_sv_wrap_validation_and_gate_checks():
    h = ctypes.c_void_p()
    assert _code(cast.sv_wrap, None, 4, cast.C128, None, ctypes.byref(h)) == -1
    assert _code(cast.sv_wrap, ctypes.c_void_p(0x1008), 4, cast.C128, None, ctypes.byref(h)) == -1  # misaligned
    # a wrapped fake pointer is never dereferenced by the validation paths below
    cast.sv_wrap(ctypes.c_void_p(0x100000), 4, cast.C128, None, ctypes.byref(h))
    m = np.eye(4, dtype=np.complex128).view(np.float64)
    mp = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    dup = (ctypes.c_int * 2)(1, 1)
    assert _code(cast.apply_gate, h, dup, 2, mp) == -1
    assert "duplicate" in cast.last_error()
    oob = (ctypes.c_int * 2)(1, 4)
    assert _code(cast.apply_gate, h, oob, 2, mp) == -1
    assert _code(cast.apply_gate, h, (ctypes.c_int * 1)(0), 7, mp) == -1
    assert _code(cast.apply_gate, h, (ctypes.c_int * 1)(0), 1, None) == -1
    t = (cast.cast_pauli_term * 1)()
    t[0].coeff, t[0].xmask, t[0].zmask = 1.0, 1 << 4, 0
    out = np.zeros(2)
    assert _code(cast.expval, h, t, 1, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -1
    cast.sv_destroy(h)


def test_gate_matrix_unknown_name():
    out = np.zeros(32)
    k = ctypes.c_int()
    assert _code(cast.gate_matrix, b"nope", None, ctypes.byref(k),
                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -1


def test_fuse_validation():
    with pytest.raises(cast.CastError):
        cast.FusedCircuit(3, [Gate("h", (3,))])
    with pytest.raises(cast.CastError):
        cast.FusedCircuit(3, [Gate("h", (0,))], k_max=7)
    with pytest.raises(cast.CastError):
        cast.FusedCircuit(3, [Gate("ry", (0,), param=0)])   # parametrised gates are bound first


def test_library_gate_matrices_match_textbook_values():
    """The library's own gate table against hand-entered textbook matrices."""
    s = 1 / np.sqrt(2)
    np.testing.assert_allclose(cast.std_matrix("h")[..., 0], [[s, s], [s, -s]], atol=1e-16)
    cx = cast.std_matrix("cx")[..., 0]
    np.testing.assert_array_equal(cx, [[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]])
    sw = cast.std_matrix("swap")[..., 0]
    np.testing.assert_array_equal(sw, [[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]])
    y = cast.std_matrix("y")
    np.testing.assert_array_equal(y[..., 1], [[0, -1], [1, 0]])
    th = 0.3
    ry = cast.std_matrix("ry", (th,))[..., 0]
    np.testing.assert_allclose(ry, [[np.cos(th / 2), -np.sin(th / 2)], [np.sin(th / 2), np.cos(th / 2)]], atol=1e-16)
    u = cast.std_matrix("u3", (np.pi / 2, 0, np.pi))[..., 0]
    np.testing.assert_allclose(u, [[s, s], [s, -s]], atol=1e-15)


def test_batch_create_validation():
    from circuits import hea_vqa, vqa_hamiltonian
    gates, P = hea_vqa(4, 1)
    H = vqa_hamiltonian(4)
    with pytest.raises(cast.CastError):
        cast.Batch([gates], [1], [P], [H])                          # n < 2
    with pytest.raises(cast.CastError) as ei:
        cast.Batch([[Gate("unitary", (0, 1, 2), matrix=np.eye(8))]], [4], [0], [H])
    assert ei.value.code == -4                                    # 3-qubit gates: unsupported
    with pytest.raises(cast.CastError):
        cast.Batch([gates], [4], [P - 1], [H])                      # param_id out of range
    with pytest.raises(cast.CastError):
        cast.Batch([gates], [4], [P], [H], mode=5)


def test_blocked_entry_points_validation():
    """The cache-blocked queries fail cleanly (no device work) on a wrong
    qubit count, a bad dtype, an index out of range or NULL arguments, and
    answer for a valid list without a GPU."""
    import ctypes

    from circuits import qft
    fc = cast.FusedCircuit(14, qft(14), k_max=4)
    npass = ctypes.c_size_t()
    assert cast._lib.blocked_info(fc.handle, 13, cast.C128, ctypes.byref(npass)) == EINVAL
    assert cast._lib.blocked_info(fc.handle, 14, 7, ctypes.byref(npass)) == EINVAL
    assert cast._lib.blocked_info(None, 14, cast.C128, ctypes.byref(npass)) == EINVAL
    assert cast._lib.blocked_info(fc.handle, 14, cast.C128, None) == EINVAL
    assert cast._lib.blocked_info(fc.handle, 14, cast.C128, ctypes.byref(npass)) == 0
    assert 1 <= npass.value < len(fc)
    first = ctypes.c_size_t()
    assert cast._lib.blocked_pass_info(fc.handle, 14, cast.C128, npass.value, ctypes.byref(first), None, None,
                                       None, None) == EINVAL
    assert cast._lib.blocked_pass_info(fc.handle, 14, cast.C128, 0, None, None, None, None, None) == 0
    assert cast._lib.apply_circuit_blocked(None, fc.handle) == EINVAL


def test_library_gate_table_matches_oracle_gates():
    """Every name of the library's gate table against the oracle's own gate
    definitions (two independent implementations), at random angles."""
    import oracle
    from circuits import Gate
    rng = np.random.default_rng(5)
    arity = {"cx": 2, "cz": 2, "cp": 2, "swap": 2, "rxx": 2, "ryy": 2, "rzz": 2}
    nparams = {"p": 1, "u3": 3, "rx": 1, "ry": 1, "rz": 1, "rxx": 1, "ryy": 1, "rzz": 1, "cp": 1}
    for name in ("id h x y z s t p u3 rx ry rz rxx ryy rzz cx cz cp swap").split():
        for _ in range(3):
            params = tuple(float(x) for x in rng.uniform(-2 * np.pi, 2 * np.pi, nparams.get(name, 0)))
            m = cast.std_matrix(name, params)
            lib = m[..., 0] + 1j * m[..., 1]
            want = oracle.gates.matrix(Gate(name, tuple(range(arity.get(name, 1))), params))
            assert lib.shape == want.shape, name
            np.testing.assert_allclose(lib, want, atol=1e-15, err_msg=name)


def test_device_byte_cap_gives_enomem():
    """CAST_MAX_DEVICE_BYTES caps what the library allocates: a state larger
    than the cap fails with CAST_ENOMEM before any device call (so this runs
    without a GPU), with the cap named in the message."""
    import subprocess
    import sys
    code = ("import ctypes, paper_2503_19894_amd as c\n"
            "h = ctypes.c_void_p()\n"
            "try:\n"
            "    c.sv_create(20, c.C128, None, ctypes.byref(h))\n"
            "    print('created')\n"
            "except c.CastError as e:\n"
            "    print(e.code, c.last_error())\n")
    env = dict(os.environ, CAST_MAX_DEVICE_BYTES=str(1 << 20))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = r.stdout.strip().splitlines()[-1]
    assert out.startswith("-2 ") and "CAST_MAX_DEVICE_BYTES" in out, out


def test_pass_shape_host_side():
    """Per-pass launch shapes live in the list's schedule per dtype; bad
    values and indices are rejected without device work."""
    import torch
    from circuits import qft
    fc = cast.FusedCircuit(20, qft(20), k_max=5)
    sched = fc.schedule(torch.complex128)
    i = next(j for j, p in enumerate(sched) if p["kernel"] == 0)
    assert fc.pass_shape(torch.complex128, i) == (-1, -1)
    fc.set_pass_shape(torch.complex128, i, 2, 10)
    assert fc.pass_shape(torch.complex128, i) == (2, 10)
    assert fc.pass_shape(torch.complex64, i) == (-1, -1)
    assert _code(fc.set_pass_shape, torch.complex128, i, 17, 10) == EINVAL
    assert _code(fc.set_pass_shape, torch.complex128, i, 0, 5) == EINVAL
    assert _code(fc.set_pass_shape, torch.complex128, len(sched), 0, 8) == EINVAL
    assert _code(cast.circuit_tune, None, fc.handle, 3, None, None) == EINVAL
    assert fc.pass_shape(torch.complex128, i) == (2, 10)
