"""MI355X-native relativistic particle-mesh step (HIP kernels behind a C ABI).

The Python layer only marshals arguments to ``libgpm.so``; importing a
symbol that needs the library raises if it has not been built.
"""
from ._lib import FIELDS, STAGES, PMError, load  # noqa: F401
from .pm import PMContext, background, make_config, query_workspace, tau_of_a  # noqa: F401
