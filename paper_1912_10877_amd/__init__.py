"""MI355X (gfx950) implementation of the state-vector hot path of Yao (arXiv:1912.10877).

The compute lives in libyao.so (HIP kernels behind the C ABI of include/yao.h); `binding`
marshals arguments to it and `autograd` wraps the reverse sweep for torch. Importing the
package loads nothing; the first binding call loads the library and fails loudly if it is
missing.
"""
__all__ = ["binding"]
