"""MI355X (gfx950) FX correlator for space VLBI: HIP kernels behind a C ABI.

  csrc/      HIP kernels and the C-ABI runtime (built into libxcorr.so)
  build.py   hipcc build of libxcorr.so
  xcorr.py   ctypes binding (argument marshalling only)

Importing the package does not load the library; `xcorr.load_library()` and
`xcorr.Correlator` do, and raise if it is not built.
"""
