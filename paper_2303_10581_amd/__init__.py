"""MI355X-native octagon filter and convex hull (arXiv 2303.10581).

Submodules:
  hullf      -- Python binding of the C-ABI library libhullf.so (HIP, gfx950):
                contexts, the filter, the hull, batched launches, the
                16-direction filter, the allocation-free filter, and the
                request loop (Server, over csrc/hullf_server.cpp)
  workloads  -- seeded synthetic inputs (Sec. 5 study cases)
  build      -- compiles libhullf.so in-tree with hipcc
Importing the package loads nothing; ``hullf`` loads the library on first use
and raises if it is missing.
"""
