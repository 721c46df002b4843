"""FP64 CPU oracle for the demagnetizing-field convolution and the LLG / atomistic
steps built on it.

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The GPU library never
imports, links or calls anything here, and nothing here imports the GPU library:
the two implementations share no code. Inputs come from ``workloads`` (seeded
random numbers only, none of the method's arithmetic).

Modules
-------
newell      cell-averaged demagnetizing tensor N(r) (Sec. II, Eq. 1, "formulas of
            Ref. [23]"): Newell f/g closed forms in the near field, moment
            expansion of the cell-pair average in the far field.
demag       H_d = -sum_j N(i-j) M_j (Eq. 1) by direct O(N^2) summation and by the
            zero-padded FFT convolution (Sec. II, Fig. 1, App. A).
llg         micromagnetic exchange (Eq. 4), LLG in Landau-Lifshitz form (Eq. 5),
            classic RK4 (Sec. III).
atomistic   spin-averaged macrocells (Eq. 9), nearest-neighbour exchange (Eq. 7),
            T = 0 stochastic LLG (Eq. 10) with Heun.
"""

# submodules are imported explicitly by their users (oracle.newell, oracle.demag, ...)
