"""MI355X (gfx950) batched EconoJax economy: HIP kernels behind a C ABI.

`binding` loads the in-tree library (libecon_mi355x.so) and marshals
arguments; `build` compiles it with hipcc.
"""
