"""Replica-exchange Metropolis simulation of an elastic bead-spring homopolymer
(Gross, Janke, Bachmann, arXiv:1107.3490) on AMD Instinct MI355X (gfx950).

The simulation itself runs in the HIP library ``libpt.so`` behind the C ABI
declared in ``include/pt.h``; :mod:`paper_1107_3490_amd.pt` is its Python
binding and :mod:`paper_1107_3490_amd.inputs` builds seeded workloads.
"""
