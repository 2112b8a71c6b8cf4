"""MI355X (gfx950) implementation of multicanonical sampling of the 3D bimodal
Edwards-Anderson spin glass with flat, 1/k and power-law weights
(Muller, Schnabel, Janke, "Nonflat Histogram Techniques for Spin Glasses").

The sampler lives in the HIP library ``libnfm.so`` (C ABI in include/nfm.h);
``nfm`` is its Python binding."""
from . import nfm  # noqa: F401
