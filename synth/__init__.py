"""Seeded synthetic inputs for the volume ray caster.

This package draws the volumes, cameras and transfer-function tables that both
the FP64 oracle (``oracle/``) and the GPU library are fed.  It holds none of the
rendering arithmetic: no ray setup, no reconstruction filter, no
classification, no compositing.  Everything here is plain NumPy driven by
``numpy.random.default_rng(seed)``, so the same call returns the same bytes on
any machine.

The paper's own data (CT tomograms in DICOM, Section 1 and Section 3) are not
available, so CT-like phantoms stand in for them: 16-bit volumes of
hundreds of slices with a large share of air, soft tissue around 0..80 HU and
bone shells of several hundred HU.
"""

from .phantoms import (  # noqa: F401
    ellipsoid_phantom_u16,
    ct_phantom_i16,
    density_grid_f32,
)
from .cameras import (  # noqa: F401
    Camera,
    ortho_axis_camera,
    orbit_camera,
    orbit_directions,
    orbit_cameras,
)
from .tfs import (  # noqa: F401
    TransferFunction,
    tf_from_points,
    TF0_POINTS,
    TF1_POINTS,
    TF3_POINTS,
    tf0,
    tf1,
    tf3,
)
from .configs import (  # noqa: F401
    config_c0,
    config_c1,
    config_c2,
    config_c3,
    config_c4_volumes,
    c4_arrivals,
    sample_pixels,
    SHADE_CT,
    SHADE_CT_HEADLIGHT,
    SHADE_C0,
)
