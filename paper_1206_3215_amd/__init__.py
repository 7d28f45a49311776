"""pst: Fourier pseudospectral time stepping on MI355X (gfx950).

The compute path lives in the HIP library ``libpst.so`` (sources under
``csrc/``); ``binding`` exposes its C-ABI entry points to Python and
``serve`` holds the continuous-batching request loop.  ``inputs`` holds the
seeded synthetic input generators, which carry none of the schemes'
arithmetic.

Nothing is imported eagerly here, so that ``inputs`` can be used without the
HIP library being present.
"""

__all__ = ["inputs", "binding", "serve"]
