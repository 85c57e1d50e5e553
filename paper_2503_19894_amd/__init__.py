"""Python binding of libcast, the MI355X fused-gate state-vector engine.

Argument marshalling only: every step of the simulation runs in the library's
HIP kernels.  The raw C entry points are re-exported under their C names
(``sv_create``, ``apply_gate``, ``fuse_circuit``, ``apply_circuit``,
``expval``, ``adjoint_grad``, ...), raising :class:`CastError` on a non-zero
status.  On top sit small conveniences: :class:`StateVector` (a torch tensor
on the GPU wrapped with ``sv_wrap``), :func:`fuse` (gate records ->
fused list) and :class:`CircuitEnergy` (``torch.autograd.Function`` whose
backward returns adjoint gradients).

Importing this package without the built library raises ImportError: there is
no fallback path.
"""
import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime libcast binds to (one runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcast.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2503_19894_amd/build.py` "
                      "(or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

C64, C128 = 1, 2
_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_double_p = ctypes.POINTER(ctypes.c_double)


class cast_gate(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("qubits", ctypes.c_int * 6), ("matrix", _c_double_p),
                ("param_id", ctypes.c_int), ("param_coeff", ctypes.c_double), ("generator", ctypes.c_int)]


class cast_fusion_opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int), ("opcount_cap", ctypes.c_double), ("zero_tol", ctypes.c_double),
                ("one_tol", ctypes.c_double), ("agglomerative", ctypes.c_int), ("multi_traversal", ctypes.c_int),
                ("cost_model", ctypes.c_int), ("cost_dtype", ctypes.c_int)]


class cast_pauli_term(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("xmask", ctypes.c_uint64), ("zmask", ctypes.c_uint64)]


#: exported symbol -> (restype, argtypes); the same list tests check against include/cast.h
SIGNATURES = {
    "cast_last_error": (ctypes.c_char_p, []),
    "pool_trim": (None, []),
    "sv_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "sv_wrap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p)]),
    "sv_destroy": (None, [ctypes.c_void_p]),
    "sv_copy_from_host": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sv_copy_to_host": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "sv_set_basis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "sv_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), _c_int_p, _c_int_p]),
    "apply_gate": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, ctypes.c_int, _c_double_p]),
    "gate_matrix": (ctypes.c_int, [ctypes.c_char_p, _c_double_p, _c_int_p, _c_double_p]),
    "fusion_opts_default": (None, [ctypes.POINTER(cast_fusion_opts)]),
    "fuse_circuit": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(cast_gate), ctypes.c_size_t,
                                    ctypes.POINTER(cast_fusion_opts), ctypes.POINTER(ctypes.c_void_p)]),
    "fused_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t), _c_double_p, _c_double_p]),
    "fused_gate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, _c_int_p, _c_int_p, _c_double_p, _c_int_p,
                                  _c_int_p, _c_double_p]),
    "apply_circuit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fused_destroy": (None, [ctypes.c_void_p]),
    "apply_circuit_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "circuit_passes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "circuit_pass_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t), _c_int_p,
                                         _c_int_p, _c_double_p, _c_double_p]),
    "circuit_pass_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_size_t, _c_int_p,
                                          _c_int_p]),
    "circuit_set_pass_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                              ctypes.c_int, ctypes.c_int]),
    "circuit_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, _c_double_p, _c_double_p]),
    "fused_pass_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _c_int_p,
                                       _c_int_p, _c_double_p, _c_double_p]),
    "apply_circuit_blocked": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "apply_circuit_blocked_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.POINTER(ctypes.c_float)]),
    "blocked_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "blocked_pass_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                         _c_int_p, _c_int_p, _c_int_p]),
    "jit_compile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, _c_int_p, _c_double_p]),
    "apply_circuit_jit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "apply_circuit_jit_timed": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]),
    "expval": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(cast_pauli_term), ctypes.c_size_t, _c_double_p]),
    "expval_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(cast_pauli_term), ctypes.c_size_t, _c_double_p]),
    "stream_scale": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_void_p]),
    "adjoint_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(cast_gate), ctypes.c_size_t, _c_double_p,
                                    ctypes.c_size_t, ctypes.POINTER(cast_pauli_term), ctypes.c_size_t,
                                    _c_double_p, _c_double_p]),
    "batch_create": (ctypes.c_int, [ctypes.c_int, _c_int_p, ctypes.c_int, ctypes.POINTER(ctypes.POINTER(cast_gate)),
                                    ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.POINTER(cast_pauli_term)), ctypes.POINTER(ctypes.c_size_t),
                                    _c_int_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_void_p)]),
    "batch_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_c_double_p), _c_double_p,
                                 ctypes.POINTER(_c_double_p)]),
    "batch_info": (ctypes.c_int, [ctypes.c_void_p, _c_int_p, ctypes.POINTER(ctypes.c_uint64), _c_double_p]),
    "batch_traffic": (ctypes.c_int, [ctypes.c_void_p, _c_double_p, ctypes.POINTER(ctypes.c_uint64)]),
    "batch_segments": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(cast_gate), ctypes.c_size_t, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]),
    "batch_destroy": (None, [ctypes.c_void_p]),
    "tuning_set": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.c_int]),
    "tuning_get": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, _c_int_p]),
    "path_cost_set": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.c_double]),
    "path_cost_get": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, _c_double_p]),
    "predict_ms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_double_p]),
    "plan_circuit": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(cast_gate), ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(cast_fusion_opts), ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_void_p), _c_int_p, _c_int_p, _c_double_p]),
    "cost_table_set": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]),
    "cost_table_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _c_double_p]),
    "adjoint_grad_batch": (ctypes.c_int, [ctypes.c_int, _c_int_p, ctypes.c_int,
                                          ctypes.POINTER(ctypes.POINTER(cast_gate)), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(_c_double_p), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.POINTER(cast_pauli_term)),
                                          ctypes.POINTER(ctypes.c_size_t), _c_int_p, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.c_int, _c_double_p, ctypes.POINTER(_c_double_p)]),
}

INIT_ZERO, INIT_PLUS, INIT_STATE = 0, 1, 2
BATCH_STEPS, BATCH_STEPS_GRAPH, BATCH_PERSISTENT_GRAPH = 0, 1, 2

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CastError(RuntimeError):  # noqa: E302
    def __init__(self, code, msg):
        super().__init__(f"libcast error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise CastError(rc, _lib.cast_last_error().decode())
    return rc


def _raw(name):
    f = getattr(_lib, name)

    def call(*args):
        r = f(*args)
        if SIGNATURES[name][0] is ctypes.c_int:
            _check(r)
        return r

    call.__name__ = name
    return call


# raw C entry points under their C names
for _name in SIGNATURES:
    if _name != "cast_last_error":
        globals()[_name] = _raw(_name)
last_error = lambda: _lib.cast_last_error().decode()  # noqa: E731


def _dptr(a):
    return a.ctypes.data_as(_c_double_p)


# --------------------------------------------------------------------- gates
#: Pauli letter codes of the rotation generators (2 bits per qubit)
_GEN = {"rx": 1, "ry": 2, "rz": 3, "rxx": 1 | (1 << 2), "ryy": 2 | (2 << 2), "rzz": 3 | (3 << 2)}


def std_matrix(name, params=()):
    """Matrix of a standard gate, built by the library (interleaved float64
    array of shape (2^k, 2^k, 2))."""
    p = np.zeros(3)
    p[:len(params)] = params
    out = np.zeros(2 * 64 * 64)
    k = ctypes.c_int()
    gate_matrix(name.encode(), _dptr(p), ctypes.byref(k), _dptr(out))
    D = 1 << k.value
    return out[:2 * D * D].reshape(D, D, 2).copy()


class GateArray:
    """cast_gate[] for a list of gate records (keeps matrices alive)."""

    def __init__(self, gates):
        self.arr = (cast_gate * max(1, len(gates)))()
        self._keep = []
        for i, g in enumerate(gates):
            cg = self.arr[i]
            cg.k = len(g.qubits)
            for j, q in enumerate(g.qubits):
                cg.qubits[j] = int(q)
            cg.param_id = int(getattr(g, "param", -1))
            cg.param_coeff = float(getattr(g, "coeff", 1.0))
            if cg.param_id >= 0:
                cg.generator = _GEN[g.name]
                cg.matrix = None
            else:
                cg.generator = 0
                if g.name == "unitary":
                    m = np.ascontiguousarray(np.asarray(g.matrix, dtype=np.complex128)).view(np.float64).copy()
                else:
                    m = np.ascontiguousarray(std_matrix(g.name, g.params)).reshape(-1)
                self._keep.append(m)
                cg.matrix = _dptr(m)
        self.n = len(gates)


def pauli_terms(terms):
    """cast_pauli_term[] from records with .coeff and .ops = ((qubit, 'X'|'Y'|'Z'), ...)."""
    arr = (cast_pauli_term * max(1, len(terms)))()
    for i, t in enumerate(terms):
        x = z = 0
        for q, p in t.ops:
            if p in "XY":
                x |= 1 << q
            if p in "YZ":
                z |= 1 << q
        arr[i].coeff = float(t.coeff)
        arr[i].xmask = x
        arr[i].zmask = z
    return arr


def fusion_options(k_max=5, opcount_cap=0.0, zero_tol=1e-14, one_tol=1e-14, agglomerative=True,
                   multi_traversal=True, cost_model=0, cost_dtype=None):
    o = cast_fusion_opts()
    o.k_max, o.opcount_cap, o.zero_tol, o.one_tol = k_max, opcount_cap, zero_tol, one_tol
    o.agglomerative, o.multi_traversal, o.cost_model = int(agglomerative), int(multi_traversal), cost_model
    o.cost_dtype = C64 if cost_dtype == torch.complex64 else C128
    return o


# --------------------------------------------------------------------- tuning
TUNING_KEYS = ("direct_min_q", "tile_bits", "direct_ipt", "direct_nt", "direct_chunk_log", "max_grid", "use_diag", "mfma_min_d",
               "mfma_grid_per_cu", "mfma_direct_min_q", "diag_unroll", "diag_max_grid", "diag_lds_table",
               "diag_order", "blocked_tile_bits", "blocked_threads", "mfma_3m_min_d", "mfma_low_tile",
               "persistent_spin_limit", "diag_run_tables", "diag_run_qubits", "diag_run_unroll", "diag_run_grid",
               "diag_run_lds", "mfma_prefetch", "diag_spread", "diag_run_reuse", "direct_rot", "direct_rot_lo",
               "direct_rot_hi", "batch_tile_bits", "batch_min_window")
PATH_COST_KEYS = tuple(f"bw{i}" for i in range(7)) + ("fl4", "fl5", "fl6", "fl_vec", "launch_ms", "seg_bw") + \
    tuple(f"seg_gate{d}" for d in range(4))
#: environment overrides (set for sweeps) take precedence over the tuning file
_ENV_OF = {"direct_min_q": "CAST_DIRECT_MIN_Q", "tile_bits": "CAST_TILE_BITS", "direct_ipt": "CAST_DIRECT_IPT",
           "direct_nt": "CAST_DIRECT_NT", "direct_chunk_log": "CAST_DIRECT_CHUNK_LOG", "max_grid": "CAST_MAX_GRID", "use_diag": "CAST_USE_DIAG",
           "mfma_min_d": "CAST_MFMA_MIN_D", "mfma_grid_per_cu": "CAST_MFMA_GRID_PER_CU",
           "mfma_direct_min_q": "CAST_MFMA_DIRECT_MIN_Q", "diag_unroll": "CAST_DIAG_UNROLL",
           "diag_max_grid": "CAST_DIAG_MAX_GRID", "diag_lds_table": "CAST_DIAG_LDS_TABLE",
           "diag_order": "CAST_DIAG_ORDER", "blocked_tile_bits": "CAST_BLOCKED_TILE_BITS",
           "blocked_threads": "CAST_BLOCKED_THREADS", "mfma_3m_min_d": "CAST_MFMA_3M_MIN_D",
           "mfma_low_tile": "CAST_MFMA_LOW_TILE"}
TUNING_FILE = os.path.join(_HERE, "tuning_gfx950.json")


def get_tuning(key, dtype=torch.complex128):
    v = ctypes.c_int()
    tuning_get(key.encode(), C128 if dtype == torch.complex128 else C64, ctypes.byref(v))
    return v.value


def set_tuning(key, value, dtype=torch.complex128):
    tuning_set(key.encode(), C128 if dtype == torch.complex128 else C64, int(value))


def apply_tuning_file(path=TUNING_FILE):
    """Applies an autotuner result (see autotune.py): launch knobs and the
    pass-cost table, skipping knobs overridden in the environment."""
    import json
    if not os.path.exists(path) or os.environ.get("CAST_NO_TUNING_FILE"):
        return False
    data = json.load(open(path))
    for dname, dt in (("c64", C64), ("c128", C128)):
        for key, value in data.get("knobs", {}).get(dname, {}).items():
            env = _ENV_OF.get(key, "")
            if os.environ.get(env) or os.environ.get(env + ("_C64" if dt == C64 else "_C128")):
                continue
            tuning_set(key.encode(), dt, int(value))
        for entry in data.get("cost", {}).get(dname, []):
            cost_table_set(dt, int(entry["k"]), int(entry["d"]), float(entry["ms_per_gamp"]))
        for key, value in data.get("path_cost", {}).get(dname, {}).items():
            path_cost_set(key.encode(), dt, float(value))
    return True


def get_path_cost(key, dtype=torch.complex128):
    v = ctypes.c_double()
    path_cost_get(key.encode(), C128 if dtype == torch.complex128 else C64, ctypes.byref(v))
    return v.value


def set_path_cost(key, value, dtype=torch.complex128):
    path_cost_set(key.encode(), C128 if dtype == torch.complex128 else C64, float(value))


def plan(n, gates, dtype=torch.complex128, k_range=(2, 6), **opts):
    """Fuses `gates` at every k_max in k_range and returns the cheapest
    (fused list, path) under the measured path costs:
    (FusedCircuit, path 0 per pass / 1 cache-blocked, k_max, predicted ms)."""
    ga = GateArray(gates)
    o = fusion_options(**opts)
    h = ctypes.c_void_p()
    path, kmax, pred = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    plan_circuit(n, ga.arr, ga.n, C128 if dtype == torch.complex128 else C64, ctypes.byref(o), int(k_range[0]),
                 int(k_range[1]), ctypes.byref(h), ctypes.byref(path), ctypes.byref(kmax), ctypes.byref(pred))
    return FusedCircuit._adopt(n, h), path.value, kmax.value, pred.value


class FusedCircuit:
    """A fused gate list owned by the library."""

    @classmethod
    def _adopt(cls, n, handle):
        """Wraps a fused list the library created (takes ownership)."""
        self = cls.__new__(cls)
        self.handle = handle
        self.n = n
        return self

    def predict_ms(self, dtype, path):
        """Predicted device time of apply_circuit (path 0) or
        apply_circuit_blocked (path 1) under the measured path costs."""
        v = ctypes.c_double()
        predict_ms(self.handle, self.n, C128 if dtype == torch.complex128 else C64, int(path), ctypes.byref(v))
        return v.value

    def __init__(self, n, gates, **opts):
        ga = GateArray(gates)
        o = fusion_options(**opts)
        h = ctypes.c_void_p()
        fuse_circuit(n, ga.arr, ga.n, ctypes.byref(o), ctypes.byref(h))
        self.handle = h
        self.n = n

    def info(self):
        nf, oc, ms = ctypes.c_size_t(), ctypes.c_double(), ctypes.c_double()
        fused_info(self.handle, ctypes.byref(nf), ctypes.byref(oc), ctypes.byref(ms))
        return {"n_fused": nf.value, "opcount": oc.value, "fusion_ms": ms.value}

    def gate(self, i, with_matrix=False):
        k, d, nb, oc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        qs = (ctypes.c_int * 6)()
        m = np.zeros(2 * 64 * 64) if with_matrix else None
        fused_gate(self.handle, i, ctypes.byref(k), qs, ctypes.byref(oc), ctypes.byref(d), ctypes.byref(nb),
                   _dptr(m) if with_matrix else None)
        out = {"k": k.value, "qubits": tuple(qs[:k.value]), "opcount": oc.value, "d": d.value,
               "active_blocks": nb.value}
        if with_matrix:
            D = 1 << k.value
            out["matrix"] = m[:2 * D * D].view(np.complex128).reshape(D, D)
        return out

    def pass_info(self, i, dtype):
        """Kernel choice and algorithmic bytes / flops of pass i on this
        circuit's n qubits in `dtype` (torch complex dtype)."""
        dt = C128 if dtype == torch.complex128 else C64
        kern, d = ctypes.c_int(), ctypes.c_int()
        b, f = ctypes.c_double(), ctypes.c_double()
        fused_pass_info(self.handle, i, self.n, dt, ctypes.byref(kern), ctypes.byref(d), ctypes.byref(b),
                        ctypes.byref(f))
        return {"kernel": kern.value, "d": d.value, "alg_bytes": b.value, "flops": f.value}

    def num_passes(self, dtype):
        """Device passes apply_circuit makes for this dtype (current knobs)."""
        dt = C128 if dtype == torch.complex128 else C64
        npass = ctypes.c_size_t()
        circuit_passes(self.handle, self.n, dt, ctypes.byref(npass))
        return npass.value

    def schedule(self, dtype):
        """The passes of apply_circuit: fused gates covered, kernel, phase
        tables of a diagonal run, algorithmic bytes and flops."""
        dt = C128 if dtype == torch.complex128 else C64
        out = []
        for i in range(self.num_passes(dtype)):
            first, count = ctypes.c_size_t(), ctypes.c_size_t()
            kern, tabs = ctypes.c_int(), ctypes.c_int()
            b, f = ctypes.c_double(), ctypes.c_double()
            circuit_pass_info(self.handle, self.n, dt, i, ctypes.byref(first), ctypes.byref(count),
                              ctypes.byref(kern), ctypes.byref(tabs), ctypes.byref(b), ctypes.byref(f))
            out.append({"first": first.value, "count": count.value, "kernel": kern.value, "tables": tabs.value,
                        "alg_bytes": b.value, "flops": f.value})
        return out

    def pass_shape(self, dtype, i):
        """(rot, chunk_log) launch shape of pass i (-1: the knob's value)."""
        dt = C128 if dtype == torch.complex128 else C64
        r, c = ctypes.c_int(), ctypes.c_int()
        circuit_pass_shape(self.handle, self.n, dt, i, ctypes.byref(r), ctypes.byref(c))
        return r.value, c.value

    def set_pass_shape(self, dtype, i, rot=-1, chunk_log=-1):
        dt = C128 if dtype == torch.complex128 else C64
        circuit_set_pass_shape(self.handle, self.n, dt, i, int(rot), int(chunk_log))

    def blocked_passes(self, dtype):
        """The cache-blocked grouping on this circuit's n qubits in `dtype`:
        one dict per HBM pass with the fused gates it covers and, for a
        segment, its tile geometry (tile_bits = 0 for an ordinary pass)."""
        dt = C128 if dtype == torch.complex128 else C64
        np_ = ctypes.c_size_t()
        blocked_info(self.handle, self.n, dt, ctypes.byref(np_))
        out = []
        for i in range(np_.value):
            first, count = ctypes.c_size_t(), ctypes.c_size_t()
            tb, w = ctypes.c_int(), ctypes.c_int()
            hq = (ctypes.c_int * 10)()
            blocked_pass_info(self.handle, self.n, dt, i, ctypes.byref(first), ctypes.byref(count), ctypes.byref(tb),
                              ctypes.byref(w), hq)
            out.append({"first": first.value, "count": count.value, "tile_bits": tb.value, "window": w.value,
                        "high_qubits": tuple(q for q in hq if q >= 0)})
        return out

    def jit_compile(self, dtype):
        """Compiles the generated kernels for `dtype` (host only); returns
        (kernel count, compile ms)."""
        dt = C128 if dtype == torch.complex128 else C64
        nk, ms = ctypes.c_int(), ctypes.c_double()
        jit_compile(self.handle, dt, ctypes.byref(nk), ctypes.byref(ms))
        return nk.value, ms.value

    def __len__(self):
        return self.info()["n_fused"]

    def __del__(self, _destroy=_lib.fused_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


# --------------------------------------------------------------------- states
class StateVector:
    """A 2^n state in a torch tensor (complex64 / complex128 on a GPU),
    wrapped for the library on the tensor's current stream."""

    def __init__(self, n, dtype=torch.complex128, device="cuda", tensor=None):
        if tensor is None:
            tensor = torch.zeros(1 << n, dtype=dtype, device=device)
            tensor[0] = 1
        assert tensor.is_cuda and tensor.is_contiguous() and tensor.numel() == 1 << n
        assert tensor.dtype in (torch.complex64, torch.complex128)
        self.tensor = tensor
        self.n = n
        self.dt = C128 if tensor.dtype == torch.complex128 else C64
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(tensor.device).cuda_stream
        sv_wrap(ctypes.c_void_p(tensor.data_ptr()), n, self.dt, ctypes.c_void_p(stream), ctypes.byref(h))
        self.handle = h

    def apply_gate(self, qubits, matrix):
        m = np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128)).view(np.float64)
        q = (ctypes.c_int * len(qubits))(*[int(x) for x in qubits])
        apply_gate(self.handle, q, len(qubits), _dptr(m))

    def apply_circuit(self, fused: FusedCircuit):
        apply_circuit(self.handle, fused.handle)

    def apply_circuit_timed(self, fused: FusedCircuit):
        """Applies the circuit and returns the device time (ms) of each pass
        of its schedule (FusedCircuit.schedule)."""
        nf = fused.num_passes(self.tensor.dtype)
        out = (ctypes.c_float * max(1, nf))()
        apply_circuit_timed(self.handle, fused.handle, out)
        return np.array(out[:nf], dtype=np.float64)

    def tune_circuit(self, fused: FusedCircuit, reps=3):
        """Measures and keeps the launch shape of each direct, matrix-core
        direct and diagonal-run pass (circuit_tune); changes this state's
        amplitudes.  Returns (ms before, ms after) of the tuned passes."""
        b, a = ctypes.c_double(), ctypes.c_double()
        circuit_tune(self.handle, fused.handle, int(reps), ctypes.byref(b), ctypes.byref(a))
        return b.value, a.value

    def apply_circuit_blocked(self, fused: FusedCircuit):
        """Applies the circuit with several fused gates per HBM pass."""
        apply_circuit_blocked(self.handle, fused.handle)

    def apply_circuit_blocked_timed(self, fused: FusedCircuit):
        """Applies the circuit cache-blocked; returns per-HBM-pass device times (ms)."""
        npass = len(fused.blocked_passes(self.tensor.dtype))
        out = (ctypes.c_float * max(1, npass))()
        apply_circuit_blocked_timed(self.handle, fused.handle, out)
        return np.array(out[:npass], dtype=np.float64)

    def apply_circuit_jit(self, fused: FusedCircuit):
        """Applies the circuit with its generated (immediate-valued) kernels."""
        apply_circuit_jit(self.handle, fused.handle)

    def apply_circuit_jit_timed(self, fused: FusedCircuit):
        """Applies the circuit with its generated kernels; per-pass device times (ms)."""
        nf = len(fused)
        out = (ctypes.c_float * max(1, nf))()
        apply_circuit_jit_timed(self.handle, fused.handle, out)
        return np.array(out[:nf], dtype=np.float64)

    def expval(self, terms):
        arr = pauli_terms(terms)
        out = np.zeros(2)
        expval(self.handle, arr, len(terms), _dptr(out))
        return complex(out[0], out[1])

    def expval_noalloc(self, terms):
        """expval with the device scratch in the library's fixed array (no
        device allocation; at most CAST_EXPVAL_NOALLOC_MAX_TERMS terms)."""
        arr = pauli_terms(terms)
        out = np.zeros(2)
        expval_noalloc(self.handle, arr, len(terms), _dptr(out))
        return complex(out[0], out[1])

    def numpy(self):
        torch.cuda.current_stream(self.tensor.device).synchronize()
        return self.tensor.cpu().numpy()

    def __del__(self, _destroy=_lib.sv_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def adjoint(init: StateVector, gates, theta, terms):
    """(energy, gradient) of <psi(theta)|H|psi(theta)> by the adjoint method."""
    ga = GateArray(gates)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    grad = np.zeros(max(1, th.size))
    e = ctypes.c_double()
    arr = pauli_terms(terms)
    adjoint_grad(init.handle, ga.arr, ga.n, _dptr(th), th.size, arr, len(terms), ctypes.byref(e), _dptr(grad))
    return e.value, grad[:th.size].copy()


class Batch:
    """Batched energies and adjoint gradients of many parametrised circuits
    (one library batch: device states, pinned matrices, optional hipGraph).

    circuits[i]: gate records of instance i (1- and 2-qubit gates),
    n_qubits[i], n_params[i], hamiltonians[i]: Pauli-term records; init[i]:
    "zero", "plus" or a StateVector of the same size and dtype."""

    def __init__(self, circuits, n_qubits, n_params, hamiltonians, dtype=torch.complex128, init=None,
                 mode=BATCH_STEPS_GRAPH):
        B = len(circuits)
        self.B = B
        self.n_params = [int(p) for p in n_params]
        self._gates = [GateArray(c) for c in circuits]
        self._terms = [pauli_terms(h) for h in hamiltonians]
        self._init = init
        nq = (ctypes.c_int * B)(*[int(n) for n in n_qubits])
        circ = (ctypes.POINTER(cast_gate) * B)(*[ctypes.cast(g.arr, ctypes.POINTER(cast_gate)) for g in self._gates])
        ng = (ctypes.c_size_t * B)(*[g.n for g in self._gates])
        npar = (ctypes.c_size_t * B)(*self.n_params)
        hp = (ctypes.POINTER(cast_pauli_term) * B)(
            *[ctypes.cast(t, ctypes.POINTER(cast_pauli_term)) for t in self._terms])
        nt = (ctypes.c_size_t * B)(*[len(h) for h in hamiltonians])
        kinds = (ctypes.c_int * B)()
        srcs = (ctypes.c_void_p * B)()
        for i in range(B):
            it = "zero" if init is None else init[i]
            if isinstance(it, StateVector):
                kinds[i], srcs[i] = INIT_STATE, it.handle.value
            else:
                kinds[i] = {"zero": INIT_ZERO, "plus": INIT_PLUS}[it]
        dt = C128 if dtype == torch.complex128 else C64
        h = ctypes.c_void_p()
        batch_create(B, nq, dt, circ, ng, npar, hp, nt, kinds, srcs, int(mode), ctypes.byref(h))
        self.handle = h

    def info(self):
        ns, items, sb = ctypes.c_int(), ctypes.c_uint64(), ctypes.c_double()
        batch_info(self.handle, ctypes.byref(ns), ctypes.byref(items), ctypes.byref(sb))
        return {"steps": ns.value, "items": items.value, "state_bytes": sb.value}

    def traffic(self):
        """Algorithmic HBM bytes of one run and its whole-state passes."""
        ab, sp = ctypes.c_double(), ctypes.c_uint64()
        batch_traffic(self.handle, ctypes.byref(ab), ctypes.byref(sp))
        return {"alg_bytes": ab.value, "state_passes": sp.value}

    def run(self, thetas):
        """thetas[i]: n_params[i] angles.  Returns (energies [B], grads list)."""
        th = [np.ascontiguousarray(t, dtype=np.float64).reshape(-1) for t in thetas]
        gr = [np.zeros(max(1, p)) for p in self.n_params]
        tp = (_c_double_p * self.B)(*[_dptr(t) for t in th])
        gp = (_c_double_p * self.B)(*[_dptr(g) for g in gr])
        e = np.zeros(self.B)
        batch_run(self.handle, tp, _dptr(e), gp)
        return e, [g[:p].copy() for g, p in zip(gr, self.n_params)]

    def __del__(self, _destroy=_lib.batch_destroy):
        if getattr(self, "handle", None):
            _destroy(self.handle)
            self.handle = None


def segments(n, gates, dtype=torch.complex128, reverse=False):
    """The segments batch_create cuts a batched instance's gate list into:
    a list of segments, each the gate indices it applies in order."""
    ga = GateArray(gates)
    cnt = ctypes.c_size_t()
    order = (ctypes.c_int * max(1, ga.n))()
    seg = (ctypes.c_int * max(1, ga.n))()
    batch_segments(n, ga.arr, ga.n, C128 if dtype == torch.complex128 else C64, int(reverse), ctypes.byref(cnt),
                   order, seg)
    out = [[] for _ in range(cnt.value)]
    for i in range(ga.n):
        out[seg[i]].append(order[i])
    return out


class CircuitEnergy(torch.autograd.Function):
    """E[b] = <psi(theta_b)|H|psi(theta_b)> for theta of shape [B, P] (or [P]);
    backward returns grad_out[b] * dE[b]/dtheta_b from the adjoint sweep done
    in forward."""

    @staticmethod
    def forward(ctx, theta, n, gates, terms, dtype=torch.complex128):
        th = theta.detach().to("cpu", torch.float64)
        flat = th.reshape(-1, th.shape[-1]).numpy()
        P = flat.shape[1]
        if flat.shape[0] > 1 and all(len(g.qubits) <= 2 for g in gates):
            # all parameter sets in one batched program
            b = Batch([gates] * flat.shape[0], [n] * flat.shape[0], [P] * flat.shape[0],
                      [terms] * flat.shape[0], dtype=dtype)
            es, gs = b.run(list(flat))
        else:
            init = StateVector(n, dtype=dtype)
            es, gs = [], []
            for row in flat:
                e, g = adjoint(init, gates, row, terms)
                es.append(e)
                gs.append(g)
        # the gradient lives where theta lives, so autograd gets it back on
        # theta's device whatever that is
        ctx.save_for_backward(torch.tensor(np.array(gs), dtype=theta.dtype).reshape(theta.shape).to(theta.device))
        return torch.tensor(np.asarray(es), dtype=theta.dtype).reshape(theta.shape[:-1]).to(theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out.unsqueeze(-1).to(g.device) * g, None, None, None, None


apply_tuning_file()
