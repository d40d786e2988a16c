"""MI355X-native multi-level ADK ionization step (Cheng & Samulyak).

The compute path is the HIP library ``libadkion.so`` built from ``csrc/``;
``adkion`` is its Python binding.  ``workloads`` draws seeded synthetic inputs.
"""
