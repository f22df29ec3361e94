"""MI355X (gfx950) Monte-Carlo BEM and dense Burton-Miller BEM library.

The compute lives in libnat_bem.so (hand-written HIP, C ABI in
include/nat_bem.h); ``nat`` is its ctypes binding."""
from . import nat  # noqa: F401
