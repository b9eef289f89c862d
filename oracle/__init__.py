"""FP64 CPU oracle of the patch-hashing zoom path (arXiv:1004.3980).

TEST INFRASTRUCTURE ONLY. A plain, slow implementation written from the
paper, used to check the HIP path: only tests/, the package smoke check and
the benchmark's CPU-baseline leg may import it. It shares no code with the
HIP library (the seeded input generator `synthdata` holds no arithmetic of
the method and is the only module both sides use).

Modules:
  imaging      degradation (Section 2.1), bicubic, patch features
               (Section 4.1), training dictionary (Section 2.1)
  lsh          Cauchy p-stable hash (Eq. hash_fn, Eq. cauchy), k-tuples and
               L tables (Section 3.2), candidate union
  lle          K nearest by exact distance, LLE weights (Eq. LinSys), HR
               synthesis (Eq. HR_Rec), overlap blend (Section 4 prior)
  backproject  error back-projection (Eq. Err_img) with the approximate cross
               bilateral filter (Section 4.3)
  pipeline     the whole path for one image
"""
from . import imaging, lsh, lle, backproject, pipeline  # noqa: F401
