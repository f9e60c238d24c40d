"""FP64 CPU oracle for the MUFFIN primal-dual reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's definitions (Sec. 2 eqs. (model), (reg), (RegAll);
Sec. 3 definition of sat and Algorithm 1) used to check the HIP path.  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library and its Python binding never do.  It shares no code with the HIP
path.
"""
from . import muffin, cnn, uob, visibility  # noqa: F401
