"""MI355X-native integral-form radiative transfer hot path (arXiv 2306.05789).

Modules are imported explicitly: `inputs` (seeded synthetic inputs, no method
arithmetic) and `rte` (ctypes binding of the HIP library librte.so)."""
