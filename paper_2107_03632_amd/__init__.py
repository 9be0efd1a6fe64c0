"""RBF-FD Laplacian stencil weights on MI355X (gfx950).

The compute path is the HIP library ``librbffd.so`` (built from ``csrc/``)
behind a C ABI; ``binding`` marshals torch tensors into it.  Importing this
package loads nothing: the library is opened on first use and its absence is
an error, never a fallback.
"""

__all__ = ["nodes", "binding"]
