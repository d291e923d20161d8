"""Plain, slow, obviously-correct CPU oracle for the PIMC transition-amplitude estimator.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import anything in this package. The product path (the HIP library and its
Python binding) never imports, calls or links it, and it imports nothing from the product.

Contents (each module cites the passage of Balaz et al., "SPEEDUP Code for Calculation of
Transition Amplitudes via the Effective Action Approach", that it follows):

* ``effective_action`` -- exact rational coefficients c_{m,k}(x) of the level-p effective
  potential for a polynomial V, by eq.(1Drec) and eq.(diagonal) in the order of Fig. 1 (Sec. 2.1).
* ``philox``           -- Philox4x32-10 counter-based generator (Salmon et al., SC'11), the
  uniform conversion and the Box-Muller normals that replace SPRNG + Box-Muller (Sec. 4.1).
* ``pimc``             -- bisection paths (Sec. 4.1), the discretized action eq.(SNp), and the
  Monte Carlo amplitude/error per bisection level (Sec. 4.1), in FP64 with math.fsum.
* ``closed_forms``     -- exact references: free kernel and Mehler kernel (Sec. 2.1 definitions),
  the exact Gaussian value of the discretized harmonic amplitude A_N^(p), low-dimensional quadrature
  of A_N^(p) for any potential, and a sinc-DVR continuum amplitude.
* ``flow``             -- FP64 affine-coupling proposal (forward, log-det, weights, analytic
  gradient) used to check the GPU flow kernels.
* ``spectrum``         -- the space-discretized evolution operator of short-time amplitudes and its
  spectrum (the paper's application, Sec. 4.2 with Fig. 3).
* ``mpt``              -- the modified Poeschl-Teller potential through the recursion in tanh(alpha x)
  (Sec. 3.3, eq.(1D-MPT), eq.(1D-MPTansatz)).
* ``general``          -- the general-potential mode: c_{m,k} as polynomials in the derivatives of V
  (Sec. 3.1/3.2).
* ``vector``           -- several coordinates (Sec. 2.2): eq.(MBrec)/(DIA) component by component and
  in the rotational invariants, paths in d dimensions, a two-dimensional DVR continuum.

Parity status of every function is stated in its module header.
"""
