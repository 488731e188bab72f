"""MI355X (gfx950) well-conditioned low-rank SDP interior-point solver.

The computation lives in the HIP library libwcsdp.so (C ABI in
include/wcsdp.h); this package only marshals arguments.  Importing the
package does not load the library; the first call does, and fails loudly
when the library has not been built.
"""
from .api import Context, SdpError, default_options, solve  # noqa: F401

__all__ = ["Context", "SdpError", "default_options", "solve"]
