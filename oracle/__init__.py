"""RLOBPCG oracle: a plain, slow, CPU FP64 implementation (numpy/scipy).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import or call anything in this package.
The HIP library never links, imports or calls it, and it shares no code,
tables or constants generator with the HIP path: the two sides each implement
the SparseStack counter spec from its written definition.

Modules
  sparsestack  SparseStack embedding S (Sec. 2.2) drawn from a counter hash,
               and the sketch S*A.
  eft          Error-free transformations and the compensated dot product
               (Ogita, Rump and Oishi 2005, "Accurate sum and dot product");
               its products run in plain C with OpenMP threads
               (eft_c.c, built by oracle/build.py) when built, else in numpy,
               with identical bits either way.
  termination  Stopping rule: tolerance (eq:est_conv_criterion) plus the two
               stagnation checks (eq:stagnation-check), Alg. rlopcg.
  rlobpcg      Alg. rlopcg (b = 1) and Alg. rlobpcg (block), including the
               one-product recurrence of eq:x-defining.
  tsqr         Stable reference SVD of a tall matrix (R factor + LAPACK SVD),
               used by checks at full size.

Every function is pinned by ``tests/test_oracle_*.py`` against facts fixed by
the paper or by mathematics (dense LAPACK SVD on small inputs, planted
spectra, exact rational arithmetic, the theory's inequalities).  Parity
unpinned: iteration counts against the paper's figures (not in its text) and
the stagnation rule's literal typeset form, for which the equation form is
implemented here and on the GPU alike.
"""

from . import eft, sparsestack, termination  # noqa: F401
from .rlobpcg import RLResult, rlobpcg, default_tau  # noqa: F401
