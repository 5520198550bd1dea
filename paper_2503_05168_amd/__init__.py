"""MI355X (gfx950) hot path of Seele (arXiv 2503.05168): preprocessing with
hybrid view-dependent filtering, tile binning with a depth-keyed radix sort,
plain and contribution-aware rasterization, and its backward pass, as HIP
kernels behind the C ABI in include/seele.h.  This package is the Python
binding: argument marshalling only."""
from ._abi import lib, SeeleError  # noqa: F401
from .pipeline import (  # noqa: F401
    GaussianTensors,
    Settings,
    Renderer,
    Frame,
    CapacityError,
    seele_preprocess,
    seele_bin_sort,
    seele_bin_sort_super,
    seele_bin_sort_ex,
    seele_bin_sort_noalloc,
    seele_preprocess_staged,
    seele_rasterize_fwd,
    seele_rasterize_fwd_super,
    seele_contrib_topk,
    seele_rasterize_fwd_counted,
    seele_rasterize_fwd_queue,
    seele_rasterize_bwd,
    SeeleRender,
    render,
    seele_hp_select,
    seele_hp_segments,
    total_tiles,
    total_super_tiles,
    pixel_count,
    split_views,
)
from .hp_build import (  # noqa: F401
    ViewDependentScene,
    build_view_dependent,
    seele_gather_gaussians,
    seele_hp_accumulate,
    seele_hp_kmeans,
    seele_hp_partition,
    seele_spatial_order,
    spatially_ordered,
)
from .prefetch import (  # noqa: F401
    PrefetchingRenderer,
    seele_load_segments,
    seele_pose_extrapolate,
    seele_resident_plan,
)
from .finetune import (  # noqa: F401
    AdamOpts,
    FineTuner,
    seele_adam_step,
    seele_flip_loss,
    seele_photometric_loss,
)
