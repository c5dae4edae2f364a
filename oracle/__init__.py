"""CPU FP64 oracle of the patch-update method.  TEST INFRASTRUCTURE ONLY:
imported by tests/, the smoke check and the CPU-baseline leg of the benchmark,
never by the GPU library."""
