"""MI355X-native semiring Datalog fixpoint engine (HIP for gfx950).

Submodules: `dlfix` (binding of the C ABI in include/dlfix.h), `autograd`
(torch.autograd.Function over it), `synth` (seeded synthetic inputs),
`build` (hipcc build of libdlfix.so).
"""
