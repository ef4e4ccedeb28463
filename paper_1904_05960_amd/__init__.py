"""MI355X-native multigrid-reduction (MGR) preconditioned flexible GMRES.

The compute path is libmgr355.so (HIP kernels for gfx950 behind the C ABI of
include/mgr355.h); `mgr355` is its Python binding.
"""
from . import mgr355  # noqa: F401
