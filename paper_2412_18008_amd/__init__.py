"""MI355X (gfx950) contraction-hierarchy construction after Wan et al.,
"Parallel Contraction Hierarchies Can Be Efficient and Scalable" (ICS 2025).

The compute path is the HIP library ``libspoch.so`` built from ``csrc/``;
this package only marshals arguments to its C ABI (``include/spoch.h``).
There is no CPU fallback: importing ``binding`` without the built library,
or calling it without a GPU, raises.
"""

__all__ = ["binding", "synth"]
