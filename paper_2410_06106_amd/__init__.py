"""MI355X (gfx950) decentralized ADMM tomography with quantized exchange.

Implements the data-parallel hot path of "Distributed Tomographic
Reconstruction with Quantization" (arXiv 2410.06106) as hand-written HIP
kernels behind the C ABI declared in include/tomoadmm.h.

Submodules (imported on demand; each needs the built library
libtomoadmm.so next to this file, see ``paper_2410_06106_amd.buildlib``):

tomoadmm   thin ctypes binding, one Python function per C entry point
admm       drivers: the plain per-node launch loop and the batched,
           graph-captured form of the ADMM iteration (Alg. 4)
autograd   differentiable projector / backprojector and the unrolled ADMM
"""

__all__ = ["build"]


def build(verbose: bool = False) -> str:
    from .buildlib import build as _build
    return _build(verbose=verbose)
