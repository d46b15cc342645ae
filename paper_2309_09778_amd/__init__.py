"""MI355X-native perceptron PW_REL compressor (arXiv 2309.09778).

The compute path is the HIP library libpwrel.so (C ABI in include/pwrel.h);
`paper_2309_09778_amd.pwrel` is its thin ctypes binding.  Submodules are
imported lazily so that the seeded generators can be used without the
library."""

__all__ = ["pwrel", "synth"]
