"""DNA KL-NMF on MI355X: HIP kernels behind a C ABI (libdna.so), thin Python binding.

``paper_1301_3389_amd.dna`` is the binding (it loads the in-tree libdna.so and
raises if it is missing); ``paper_1301_3389_amd.synth`` holds the seeded input
generators.  Importing the package itself loads neither.
"""
