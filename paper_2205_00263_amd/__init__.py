"""MI355X-native batched back-substitution engine for MN-BaB (arXiv 2205.00263).

The compute path is the HIP library libmnbab.so (include/mnbab.h); this
package is its Python binding.  Importing it does not load the library; the
first call does, and fails loudly if the library has not been built.
"""
from .api import (VARIANTS, KernelTimer, Net, Problem, Server, get_kernel_variants, mnc_to_csr, relu_hull, split_costs,  # noqa: F401,E501
                  set_index, set_kernel_variants, use_torch_plumbing)
from ._lib import MnbError, lib  # noqa: F401
