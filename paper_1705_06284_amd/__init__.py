"""MI355X-native FFT polyspectrum estimator (Watkinson et al. 2017, arXiv:1705.06284).

The compute path lives in the HIP shared library ``libbispec.so`` built from
``csrc/``; ``binding`` wraps its C ABI.  ``synth`` draws seeded synthetic
input fields and imports nothing else from this package, so it can be used
without the GPU library.  Importing the package itself loads nothing.
"""
