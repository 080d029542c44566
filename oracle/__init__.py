"""CPU oracle for the PEPS einsumsvd / boundary-contraction library.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64/complex128
NumPy implementation of what the GPU library computes, written from the paper
(Pang et al., "Efficient 2D Tensor Network Simulation of Quantum Systems",
SC20).  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  It shares no code with the GPU path: the
only common dependency is the ``synth`` module, which draws seeded inputs and
holds none of the method's arithmetic.

Modules
-------
sketch      counter-based sketch generator (SplitMix64 output function)
rsvd        explicit truncated einsumsvd (definition) and randomized SVD
            on an implicit operator (Alg. 4)
network     the implicit operators of the boundary zip-up step and of the
            two-column pair network
bmps        zip-up row absorption (Alg. 3) and boundary-MPS norm (Alg. 2),
            with cached environments (Sec. IV-B)
energy      expectation values by cached strips and the uncached full
            contraction per term (Eq. 5)
ite         QR-SVD two-site update (Alg. 1, Eq. 4) and TEBD sweeps (Sec. II-D)
statevector brute-force state vectors, gates (Eqs. 1-2), norms and energies
"""
