"""MI355X (gfx950) auxiliary-problem solver of the Difference Potentials Method.

The compute path is libdpm.so (HIP kernels behind the C ABI of include/dpm.h); `api` is its
Python binding.  Importing the package does not load the library: `api` functions load it on
first use and raise if it has not been built.
"""
