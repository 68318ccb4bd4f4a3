"""MTGP (Mersenne Twister for Graphic Processors) on AMD Instinct MI355X.

- `paper_1005_4973_amd.mtgp`   : Python binding of the C ABI (include/mtgp.h)
- `paper_1005_4973_amd.inputs` : seeded synthetic parameter sets and workloads
- `paper_1005_4973_amd.build`  : in-tree hipcc build of libmtgp.so

The binding is imported lazily so that the input recipes can be used without
torch or a GPU.
"""
