"""Seeded, synthetic inputs shared by the HIP path, the oracle and the tests.

This package holds no arithmetic of the propagation method itself: it only
builds lattices, gate lists (generator bitmasks plus angles) and seeded random
Pauli sets.  Every consumer receives plain integer / float arrays.

Bit layout used everywhere: a Pauli string on n <= 128 qubits is the pair of
bitmasks (x, z), each two little-endian 64-bit words; qubit q lives at word
q >> 6, bit q & 63.  Single-qubit letters: I=(0,0), X=(1,0), Y=(1,1), Z=(0,1).
"""

from .lattice import Lattice, eagle_127, heavy_hex_21, star_graph, ball, chain  # noqa: F401
from .circuit import (  # noqa: F401
    pauli_words, words_to_letters, kicked_ising_step, kicked_ising_circuit,
    single_pauli_term, GateList,
)
from .synth import splitmix64, random_pauli_set, random_observables, random_gates  # noqa: F401
