"""FP64 CPU oracle for the flux-limited-diffusion radiation-energy step.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here; the
product path (the HIP library and its binding) never does, and shares no code
with it.  See ``oracle.fld`` for what each function follows in the paper
(Moens et al. 2022, "Radiation-hydrodynamics with MPI-AMRVAC: flux-limited
diffusion").
"""
from .fld import *  # noqa: F401,F403
from .fld import __all__  # noqa: F401
from .moments import *  # noqa: F401,F403,E402
from . import moments as _moments  # noqa: E402

__all__ = list(__all__) + list(_moments.__all__)
from .imex import *  # noqa: F401,F403,E402
from . import imex as _imex  # noqa: E402

__all__ = list(__all__) + list(_imex.__all__)
from .aniso import *  # noqa: F401,F403,E402
from . import aniso as _aniso  # noqa: E402

__all__ = list(__all__) + list(_aniso.__all__)
from .bc import *  # noqa: F401,F403,E402
from . import bc as _bc  # noqa: E402

__all__ = list(__all__) + list(_bc.__all__)
from .multigrid import *  # noqa: F401,F403,E402
from . import multigrid as _multigrid  # noqa: E402

__all__ = list(__all__) + list(_multigrid.__all__)
from .dirichlet import *  # noqa: F401,F403,E402
from . import dirichlet as _dirichlet  # noqa: E402

__all__ = list(__all__) + list(_dirichlet.__all__)
