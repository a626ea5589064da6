"""CPU FP64 oracle for the MQS surface-integral RL extractor.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it, links it or reads anything it writes.

It is a plain, slow, obviously-correct dense implementation written from the
paper (Zhu, Chen & Yang, "An SIE Formulation with Triangular Discretization
and Loop Analysis for Parameter Extraction of Arbitrarily Shaped
Interconnects"):

* ``mesh``      -- edges, modified RWG functions (Sec. II-C, Eq. RWG/ExpandJ),
                   Gram matrix of the basis (second term of Eq. Zb).
* ``integrals`` -- the triangle-pair integrals of the 1/|r-r'| kernel
                   (first term of Eq. Zb, static Green's function
                   Eq. StaticGF), both surfaces integrated numerically:
                   Sauter-Schwab cubature on touching pairs, adaptive
                   product rules elsewhere (C helper csrc/pairs.c).
* ``circuit``   -- circuit graph, spanning tree, fundamental loops and the
                   loop matrix A (Sec. III, Eqs. VolT, CurT, LoopVandI,
                   FinalME).
* ``pfft``      -- the four pFFT steps of Sec. IV-B (Eqs. Projection, FFTCal,
                   interpolation, Lb), written as explicit sparse matrices
                   and a plain numpy FFT convolution.
* ``solve``     -- dense Z_l = A Z_b A^T, dense LU, port admittance and R/L
                   extraction (Sec. V), the preconditioner of Eq. Precond as a
                   dense inverse, and a plain restarted GMRES.
* ``mlp``       -- FP64 forward/backward of the learned correction network.

Every function cites the passage it follows.  Readings of passages the paper
leaves open are listed in the design notes of the repository.
"""
