"""MI355X (gfx950) 3D delay-and-sum: C-ABI HIP library and its Python binding.

``paper_2606_13259_amd.das`` holds the binding (``Plan``, ``DASFunction`` and
the ``das_*`` entry points); ``paper_2606_13259_amd.metrics`` the image-quality
measures; ``paper_2606_13259_amd.build`` compiles the library.  Importing this
package loads nothing; the first call into ``das`` loads the library and
raises if it has not been built.
"""
__all__ = ["das", "metrics", "build"]
