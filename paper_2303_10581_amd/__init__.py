"""MI355X-native octagon filter and convex hull (arXiv 2303.10581).

Submodules:
  hullf      -- Python binding of the C-ABI library libhullf.so (HIP, gfx950)
  workloads  -- seeded synthetic inputs (Sec. 5 study cases)
  serve      -- request loop with continuous batching
Importing the package loads nothing; ``hullf`` loads the library on first use
and raises if it is missing.
"""
