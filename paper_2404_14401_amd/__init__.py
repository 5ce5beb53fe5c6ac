"""MI355X (gfx950) split-step Gross-Pitaevskii hot path (arXiv:2404.14401).

``gpe`` binds the C ABI of ``libgpe.so`` (include/gpe.h); ``workloads`` holds the
seeded synthetic inputs; ``autograd`` wraps the adjoint as a torch.autograd.Function.
"""
