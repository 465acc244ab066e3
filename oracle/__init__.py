"""Oracle: a plain, slow, FP64 CPU implementation of the hierarchically
deflated CG hot path, written from the paper's definitions.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import,
call or execute anything in this package; only the tests, the smoke check and
the benchmark's CPU-baseline leg do.  It shares no code with the HIP path:
both sides take the same seeded inputs from ``synth`` and nothing else.

Modules
-------
geometry  lattice indexing, checkerboards, embedding of half-fields
gamma     Euclidean gamma matrices (chiral basis) and chiral projectors
dwf       Wilson hop, fifth-dimension operator, M_pc, M_pc^dagger, H
cg        textbook conjugate gradients
blocks    block aggregation, Gram-Schmidt, project / promote
coarse    little Dirac operator: brute force and the Fourier trick, coarse CG
hdcg      Q, P_L, P_R, M_IRS, generalised PCG (A-DEF2, BNN), defect correction
precision 16-bit (bfloat16) rounding; H and M_IRS with 16-bit field storage
subspace  rational-filter subspace: multi-shift CG, partial fractions, wall noise
ldop      second deflation level of the coarse operator: global vectors, the
          pre-diagonalised third level, deflated CG
"""
