"""FP64 CPU oracle for the sketch-powered power method (Chenakkod & Derezinski,
"Accelerating Power Method with Fast Sketching for Stronger Low-Rank
Approximation", arXiv 2605.09755).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the GPU path: the sketch hash, the Gaussian transform,
the power loop, the orthonormalisation and the finishers are all written here
again, plainly, in NumPy/SciPy double precision.

Modules
-------
philox      Philox4x32-10 counter-based generator (Salmon et al., SC'11).
sketch      sparse sign (CountSketch-type) sketch S, Gaussian Omega; Lemma 3.2(2).
methods     Algorithm 1 (range finder), the randomised SVD finisher (Section 2,
            "Sketch-Powered Low-Rank Factorization" paragraph), Algorithm 2
            (generalised Nystrom low-rank factorisation) and Algorithm 3 (PSD
            Nystrom).
evaluate    error norms used to judge results (Frobenius / spectral residuals,
            optimal tails by Eckart-Young).
theory      Definition 3.1 (regularised spectral approximation) measured by
            brute force, for checking Lemma 3.3 and Theorem 3.5 on tiny inputs.

Parity status
-------------
* philox: the bit stream is "parity unpinned" against an external known-answer
  vector (none ships with the paper, which does not fix a generator).  Its
  outputs are pinned only through statistical properties (uniformity, sign
  balance, stream independence) in tests/test_oracle_generators.py.
* everything else is pinned by the tests named in each function's docstring.
"""
from . import philox, sketch, methods, evaluate, theory  # noqa: F401
