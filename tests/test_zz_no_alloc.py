"""expval_noalloc (device scratch in the library's fixed array, for callers
that cannot allocate) against expval on the same states: two calls in a row,
the second with a smaller state and fewer terms, both dtypes; the limit on
the term count is an argument error."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_2503_19894_amd as cast  # noqa: E402
from circuits import PauliTerm, random_state, vqa_hamiltonian  # noqa: E402

MAX_TERMS = 4096   # CAST_EXPVAL_NOALLOC_MAX_TERMS


def _terms(n, extra, seed):
    """The VQA Hamiltonian plus `extra` random Pauli strings, some x masks
    repeated more than eight times (several passes for one x mask)."""
    rng = np.random.default_rng(seed)
    terms = vqa_hamiltonian(n)
    for i in range(extra):
        if i % 3 == 0:
            ops = ((0, "X"), (int(rng.integers(1, n)), "Z"))   # x mask {0}, many z masks
        else:
            qs = rng.permutation(n)[: rng.integers(1, 6)]
            ops = tuple((int(q), "XYZ"[rng.integers(3)]) for q in qs)
        terms.append(PauliTerm(float(rng.normal()), ops))
    return terms


def _noalloc(sv, terms):
    arr = cast.pauli_terms(terms)
    out = np.zeros(2)
    rc = cast._lib.expval_noalloc(sv.handle, arr, len(terms), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, cast.last_error()
    return complex(out[0], out[1])


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64], ids=["c128", "c64"])
def test_expval_noalloc_matches_expval(dtype):
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    for n, extra, seed in ((18, 120, 1), (9, 10, 2)):   # second call: smaller state, fewer terms
        psi0 = random_state(n, seed=seed, workload=11)
        terms = _terms(n, extra, seed)
        sv = cast.StateVector(n, tensor=torch.tensor(psi0, dtype=dtype, device="cuda"))
        want = sv.expval(terms)
        got = _noalloc(sv, terms)
        print(f"n={n} terms={len(terms)} {dtype}: expval {want:.15g} noalloc {got:.15g}", flush=True)
        # same kernels, same scratch sizes, same reduction order
        assert got == want
        scale = sum(abs(t.coeff) for t in terms)
        assert abs(got - oracle.expval(psi0, terms)) <= tol * scale


def test_expval_noalloc_term_limit():
    n = 6
    sv = cast.StateVector(n, dtype=torch.complex128)
    terms = [PauliTerm(1.0, ((0, "Z"),))] * (MAX_TERMS + 1)
    arr = cast.pauli_terms(terms)
    out = np.zeros(2)
    rc = cast._lib.expval_noalloc(sv.handle, arr, len(terms), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == -1 and "scratch" in cast.last_error()
    # exactly at the limit: accepted, <0|Z_0|0> = 1 per term
    assert _noalloc(sv, terms[:MAX_TERMS]) == complex(MAX_TERMS, 0.0)
