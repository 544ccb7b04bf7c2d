"""CPU oracle of the EconoJax economy and of its policy / PPO learner.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the GPU
library (paper_2410_22165_amd) and never imports it.
"""
