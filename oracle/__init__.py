"""FP64 CPU oracle for the per-frame keyframe depth update (DeepFusion, Sec. II).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The GPU library never calls it, and this package imports nothing from the GPU
library; the only code both sides share is the seeded input generator
``kfsynth``, which holds none of the method's arithmetic.

The oracle is written for a reader holding the paper, in the paper's order:

* ``geometry``  - relative pose, projection pi(K T_C1W T_WC0 rho(x, d)) of the
  photometric error (Sec. II-B), epipolar constants.
* ``stereo``    - texture gate, epipolar search over equally spaced samples with
  a five-point (or 5x5) SSD, interpolation between two steps, the finite
  difference Jacobian and the variance (J^T J)^-1 of eq. (semi), the
  inverse-depth filter and the conversion to log space (Sec. II-B).
* ``fusion``    - the cost c(d, s) = c_semi + c_net + c_grad with Huber on every
  term (Sec. II-C), its normal equations on the 5-point grid, a direct sparse
  solve, Jacobi-preconditioned CG, and Gauss-Newton alternating between depth
  and scale; plus a converged mode giving the unique minimiser.
* ``pipeline``  - keyframe state: set prior, fuse frame, read depth; the
  keyframe rule (Sec. II); the search of disjoint pixel blocks on a pool.
* ``priors``    - the network's outputs at its own resolution resampled to the
  keyframe, with the focal-length log-depth shift (Sec. II-A).

Where the paper is silent or ambiguous a reading is taken (R1 ... R21); each
function names the readings it follows, and the design notes list them all.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force or independent library routines (the
texture gate, the bilinear sampler at fractional points and the direction of
the sub-pixel step included); no function is "parity unpinned".
"""

from . import geometry, stereo, fusion, pipeline  # noqa: F401
from .stereo import StereoParams  # noqa: F401
from .fusion import SolverParams, PriorMaps, SemiMeasurements  # noqa: F401
from .pipeline import OracleKeyframe  # noqa: F401
