"""MI355X checkpoint-image engine: dump and restore of device allocations as
verified images (CRIUgpu, arXiv 2502.16631, section 3.1). The compute path is
libmickpt.so (HIP for gfx950); see mickpt.py for the binding."""
from . import mickpt  # noqa: F401
