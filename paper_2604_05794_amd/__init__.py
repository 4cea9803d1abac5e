"""MI355X-native fusion-patch multi-view direction optimisation.

The compute path is libfusedir.so (HIP kernels for gfx950 behind the C ABI
in include/fusedir.h); ``native`` is its ctypes binding.  Importing this
package loads nothing; the first call into ``native`` loads the library and
raises if it has not been built.
"""

__all__ = ["native"]
