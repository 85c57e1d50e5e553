"""Seeded synthetic workloads: gate lists, parameter sets, Pauli sums and input
states.  This package holds input data only: gate *names*, target qubits, angles
and (for Haar-random gates) the unitary itself, which is part of the input.  It
computes no gate matrix from angles and applies nothing to a state; the oracle
and the GPU library each build gate matrices with code of their own."""
from .spec import Gate, PauliTerm, PARAMETRISABLE, GATE_ARITY
from .generators import (random_state, random_state_torch, plus_state_amp, rqc_u3_cx, qft,
                         dense_haar_layers, haar_unitary, hea_vqa, vqa_hamiltonian, vqa_thetas,
                         tfim_trotter, tfim_fields, partition_sizes, gate_sweep, iqp, ala, qvc, hes,
                         FAMILIES)
