"""Visibility index map and projective data association (Sec. 7).

Sec. 7 predicts which live surfels are visible by rendering them into an
index map at the depth resolution, and takes the corresponded pairs P of the
data term from that rendering (the paper defers the rule to Guo et al. 2017).

Readings taken here:
* surfels are rendered as unsized points (as Sec. 6.1 renders its index map),
  at 1x resolution, the nearest z winning, ties to the lower surfel index;
  every surfel is rendered (there is no confidence at this boundary);
* surfel i corresponds to pixel u_i it projects to iff it won u_i in the index
  map, u_i has a depth normal, |v_i - V(u_i)| < corr_dist and
  n_i . N(u_i) > corr_normal;
* the map is re-rendered and P re-associated at every Gauss-Newton iteration;
* with splats (the surfels as opaque discs of their radius, Sec. 7), P is
  taken per pixel: every pixel with a normal pairs with the surfel that won
  it, under the same gates on the surfel's centre and normal, so a surfel can
  hold several pairs (replica32.splat_index_map states the rendering).

All of these are integer decisions, taken by `replica32` on the FP32-rounded
live surfels.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import replica32


@dataclasses.dataclass
class DepthFrame:
    depth: np.ndarray          # (H,W) float32 as given
    N32: np.ndarray            # (H,W,3) float32 normal map (decisions)
    nvalid: np.ndarray         # (H,W) bool


def prepare_depth(depth: np.ndarray, cam, edge_gate: float) -> DepthFrame:
    N32, ok = replica32.normal_map(depth, cam, edge_gate)
    return DepthFrame(np.asarray(depth, dtype=np.float32), N32, ok)


def associate(v_live: np.ndarray, n_live: np.ndarray, valid: np.ndarray,
              frame: DepthFrame, cam, corr_dist: float, corr_normal: float):
    """Index map (H,W; -1 = empty), correspondence mask over surfels and the
    pixel (ux, uy) of every surfel."""
    v32 = v_live.astype(np.float32)
    n32 = n_live.astype(np.float32)
    I = replica32.index_map(v32, cam, valid)
    m, ux, uy = replica32.correspondence(v32, n32, I, frame.depth, frame.N32, frame.nvalid,
                                         cam, corr_dist, corr_normal, valid)
    return I, m, ux, uy


def associate_splats(v_live: np.ndarray, n_live: np.ndarray, radius: np.ndarray, valid: np.ndarray,
                     frame: DepthFrame, cam, corr_dist: float, corr_normal: float):
    """Splat index map and its pairs (surfel, pixel x, pixel y), row-major."""
    v32 = v_live.astype(np.float32)
    n32 = n_live.astype(np.float32)
    I = replica32.splat_index_map(v32, n32, radius, cam, valid)
    k, ux, uy = replica32.splat_pairs(v32, n32, I, frame.depth, frame.N32, frame.nvalid, cam, corr_dist,
                                      corr_normal)
    return I, k, ux, uy
