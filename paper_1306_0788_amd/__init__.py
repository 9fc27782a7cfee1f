"""MI355X-native two-component Shan-Chen lattice Boltzmann fluid coupled to
off-lattice point particles (arXiv 1306.0788).

``paper_1306_0788_amd.lbmd`` is the Python binding of the C-ABI library
``liblbmd.so`` (HIP, gfx950); ``paper_1306_0788_amd.workloads`` holds the
seeded synthetic inputs.  Importing the package loads nothing; the binding
loads the library on first use and raises if it has not been built.
"""
