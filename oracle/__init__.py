"""Plain FP64 CPU oracle for fixed-precision randomized QB (randQB_EI / randQB_FP).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  The GPU library never calls it and
shares no code with it: the oracle re-derives every step from the paper
(Yu, Gu, Li: "Efficient randomized algorithms for the fixed-precision low-rank
matrix approximation", arXiv 1606.09402) with NumPy/SciPy in float64.

Modules
-------
rng      counter-based Gaussian test matrix (Philox4x32-10 + Box-Muller with
         elementary functions built from IEEE +,-,*,/ only), bit-specified.
randqb   Algorithm 1 framework, Algorithm 2 (randQB_EI), Algorithm 3 / 4
         (randQB_FP with the power scheme, P >= 0), the fixed-rank randQB special
         case, a one-sided Jacobi SVD and the SVD-optimal rank used as pins.
lowp     bfloat16 rounding for the precision form.
svd      the approximate SVD from a QB factorisation (eq. (3)).
trqrcp   trQRCP (randomized QR with column pivoting) driven by the indicator (Remark 3.2).
diff     fixed-rank randQB_FP as a differentiable map A -> (Q, B) in float64
         torch CPU autograd (reference gradient for the differentiation form).
"""
