"""MI355X-native hybrid VDIA + VBR + CSR sparse products (libsable) and its Python binding.

The binding (``paper_2407_00829_amd.sable``) loads ``libsable.so`` lazily: importing it does
not touch the GPU, and a missing library raises on first use.
"""
