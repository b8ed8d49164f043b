"""Plain FP64 CPU oracle for group-wise Naive Bayes malware detection
(Sahay & Chaudhari, "An Efficient Detection of Malware by Naive Bayes
Classifier Using GPGPU", 2019).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
definition that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with the HIP path.

Modules
  nb         training counts, Laplace-smoothed log tables, joint log-likelihood
             scores, decision rule and posteriors (section 4, posterior equation
             and the malware/benign decision that follows it)
  groups     size-group model validity and fallback routing (section 4, the
             fewer-than-six-files rule and the next-group fallback)
  select     per-group top-k feature selection by the normalised malware-benign
             occurrence difference, the feature gather, and the model trained
             on the selected features (section 3 feature selection; section 4,
             each group trained and tested on its top-k features)
  (nb also holds the Gaussian variant: exact moment sums, mean/variance
             with the variance floor, the density and its expanded weight form)
  precision  reduced-precision mirrors: BF16 and FP32 round-to-nearest-even
             from FP64, FP8-e4m3 quantisation of counts, certified label bands

Parity status: every function here is pinned by the not-gpu tests (worked
example, exact rationals, library cross-checks, invariants); none is
"parity unpinned".  The paper's own empirical results (about 87% accuracy,
up to 200x speed-up) need its dataset and hardware and are not reproduced.
"""
from . import nb, groups, precision, select  # noqa: F401
