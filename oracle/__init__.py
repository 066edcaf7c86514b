"""Reference oracle for the HEOM Liouvillian hot path (arXiv 2306.07522).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
implementation of what the GPU library computes.  It exists so that the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` can check the GPU path against the paper.  Nothing in the
product path imports, links or executes it, and it imports nothing from
the product package: the two share no code.

Modules
-------
exponents   bath correlation exponents (Methods: "Fermion correlation function
            with Lorentzian spectral density", "Boson correlation function
            with Drude-Lorentz spectral density") and the Pade
            parameters kappa, zeta built two independent ways.
hierarchy   enumeration of auxiliary density operators (ADOs) and the
            hierarchy dictionary (Results, eq:HEOM and the truncation
            paragraph after it).
liouvillian explicit Kronecker-product assembly of the HEOM Liouvillian
            superoperator (HEOMLS) M as a sparse matrix (eq:HEOM and the
            superoperators A, B, C, D, P_s defined right after it).
solvers     RK4 propagation, stationary state (direct sparse LU), and the
            frequency-domain spectra (Methods: "Numerical computation of
            the spectrum").
nn          the learned block preconditioner's MLP, forward and backward,
            in FP64 and in FP32 with BF16-rounded operands.
spmv_c      a plain C OpenMP CSR SpMV used only to time the oracle's apply
            on all host cores.

Readings of points the paper leaves open are stated where they are used;
the important ones are: fermionic ADOs are antisymmetric in their
exponent indices and stored once per set in descending index order; the
parity projector's level is that of the ADO it acts on; the stationary
state replaces the (0,0) element equation of the reduced density operator
by the trace condition.
"""
