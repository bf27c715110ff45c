"""MI355X (gfx950) implementation of the Kronecker-product path-query
algorithm of Shemetova et al. (arXiv 2103.14688): index creation for
context-free and regular path queries as hand-written HIP kernels behind a C
ABI (include/cfpq.h).

  rsm   -- query compiler: regular expressions and grammars to RSM arrays
  cfpq  -- thin binding of the C ABI (libcfpq.so); no CPU fallback
  build -- hipcc build of libcfpq.so
"""
from . import rsm  # noqa: F401

__all__ = ["rsm", "cfpq", "build"]
