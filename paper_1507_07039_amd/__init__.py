"""MI355X-native PANDA message passing (arXiv 1507.07039).

The compute path is the HIP library ``libpanda.so`` built from ``csrc/``;
``panda`` is its thin Python binding (argument marshalling only).
"""
