"""Red-green weighted minwise hashing on MI355X (arXiv 1602.08393).

``paper_1602_08393_amd.wmh`` binds the C-ABI library ``libwmh.so`` (HIP kernels for gfx950);
``paper_1602_08393_amd.synth`` builds seeded synthetic inputs.  Importing the package loads
neither; the library is loaded on first use and raises if it has not been built.
"""
