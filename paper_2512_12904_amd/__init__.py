"""HQC decryption core for AMD Instinct MI355X (gfx950).

The compute path is the C-ABI library libhqc_gpu.so (hand-written HIP,
declared in include/hqc_gpu.h); `paper_2512_12904_amd.hqc` is its thin
Python binding (argument marshalling onto torch device tensors and streams).
`paper_2512_12904_amd.synth` draws seeded synthetic inputs.
"""
