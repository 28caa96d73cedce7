"""Filtered Lanczos procedure on MI355X (gfx950).

The compute path is the HIP library ``libflp.so`` (built by
``paper_2409_15053_amd.build``) behind the C ABI of ``include/flp.h``;
``paper_2409_15053_amd.flp`` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
__all__ = ["flp", "inputs", "build"]
