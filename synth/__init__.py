"""Seeded synthetic inputs (geometry, events, seeds) shared by the tests, the
benchmark and the smoke check.  Input side only: no part of the method."""
from .workloads import (BARREL, DISK, KAPPA, CleaningConfig, EventRecipe, FindConfig, Layer, SeedingConfig,
                        Workload,
                        barrel_endcap, batched_uneven, cms_like, dense, layer_arrays,
                        small_barrel, stereo_layer, Region, five_regions,
                        MaterialMap, material_map, barrel_material, cms_like_material,
                        PION_MASS, FieldMap, solenoid_field, barrel_endcap_field)
from .events import Event, EventBatch, generate, generate_event, make_batch, simulate_tracks
