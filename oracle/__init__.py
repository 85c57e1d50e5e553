"""Plain, slow, obviously-correct CPU FP64 oracle for the state-vector hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or run anything in this package.
It shares no code with the GPU library (``paper_2503_19894_amd``) and never
imports it.

What it computes (each function cites the passage it follows):
  * gate application, Eq. 3 (C, ``sv_oracle.c``), unfused, gate by gate;
  * standard gate matrices (``gates.py``);
  * Pauli-sum expectation values by applying Pauli factors as 1-qubit gates;
  * adjoint-method gradients (Jones & Gacon 2020), central finite differences
    and the parameter-shift rule (``sim.py``).
Pins for every function live in ``tests/test_oracle_*.py``.
"""
from .sim import (apply_gate, run_circuit, expval, adjoint_grad, finite_diff_grad,
                  param_shift_grad, energy, apply_gate_groups, group_index, inner)
from . import gates
