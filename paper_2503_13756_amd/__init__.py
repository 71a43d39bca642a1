"""MI355X (gfx950) rigid alignment of images in sliced 2-Wasserstein distance.

The compute path is libswalign.so (HIP kernels behind the C ABI of
include/swalign.h); `api` binds it with torch tensors as device memory.
Importing this package does not load the library; `api` loads it on first
use and raises if it has not been built."""

__all__ = ["api", "build"]
