"""CPU oracle for the matching-pursuit correlation path -- TEST INFRASTRUCTURE.

This package is a plain, slow, FP64 (numpy/scipy) statement of what the GPU
library computes, written from the paper (Kim, Park, Hong, No, Chung, "Fast
Correlation Computation Method for Matching Pursuit Algorithms in Compressed
Sensing", arXiv 1205.4139).  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the library never does, and it
shares no code with the HIP path.

Modules
-------
unitary    the two unitary classes (Sec. I; constraints of Sec. I, Thm 2-1),
           dense rows of Phi = S_Omega U, and transform-tier adjoint/forward.
problem    y = Phi x + eta, eq. (CSbasic), with the stated SNR reading.
fastcorr   the correlation kernel vector c (definition after eq. (kernelsum)),
           the permutations P_lambda (Thm 2-1, Sec. III-B storage
           subsections) and the fast correlation of eqs. (kernelsum) and
           (kernelsumOMP).
mpa        OMP (Algorithm 1.1) with conventional or fast correlation, plus the
           SP and CoSaMP readings (cited, not defined, in the paper: parity
           unpinned by the paper for their halting and pruning details).
costmodel  the flop model of Table I and the two worked numbers of Sec. IV.
certify    selection-gap bookkeeping used to decide which instances admit
           bit-exact support parity at a given correlation precision.
"""
from . import unitary, problem, fastcorr, mpa, costmodel, certify  # noqa: F401
from .unitary import (fourier_rows, hadamard_rows, sensing_matrix, Operator,  # noqa: F401
                      DenseOperator, TransformOperator, make_operator, wht)
from .problem import measure  # noqa: F401
from .fastcorr import kernel_vector, permute, fast_correlation  # noqa: F401
from .mpa import omp, sp, cosamp, argmax_excluding, topk  # noqa: F401
