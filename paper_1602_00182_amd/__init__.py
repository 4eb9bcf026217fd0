"""MI355X-native non-polynomial (MQ-RBF perturbed) WENO5 finite-volume solver.

The compute path is the HIP library ``libnpweno.so`` (built from ``csrc/``) behind the C ABI
declared in ``include/npweno.h``; ``binding`` marshals arguments to it.
"""
