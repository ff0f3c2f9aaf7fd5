"""Seeded synthetic inputs shared by the reconstruction library's tests and
benchmark and by the FP64 oracle's tests.

This package holds input generation only (workload sizes, phantoms, channel
data, random tensors); it contains none of the reconstruction arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .configs import Scan, TINY, PAPER, WORKLOADS, describe, uniform_delays, delays_from_sos_offsets
from .phantoms import (SosPhantom, Blobs, make_sos_phantom, make_blobs, render_ip, sos_grid_truth,
                       free_node_mask, axis)
from .channels import channel_data, travel_times, point_source_data
from . import nf  # noqa: F401


@dataclass
class ScanInputs:
    scan: Scan
    phantom: SosPhantom
    blobs: Blobs
    S: np.ndarray            # [n_elem][n_t] float32 channel data
    delays: np.ndarray       # [M] float64, mm
    sos_true: np.ndarray     # [G][G] float64, phantom at SOS node centres
    mask: np.ndarray         # [G][G] uint8, 1 = free node
    ip_true: np.ndarray      # [ny][nx] float64 clean initial pressure


def make_inputs(scan: Scan, seed: int | None = None, with_channels: bool = True,
                snr_db: float | None = None) -> ScanInputs:
    rng = np.random.default_rng(scan.seed if seed is None else seed)
    ph = make_sos_phantom(scan, rng)
    blobs = make_blobs(scan, rng)
    S = channel_data(scan, ph, blobs, rng=rng, snr_db=snr_db) if with_channels else None
    return ScanInputs(scan=scan, phantom=ph, blobs=blobs, S=S,
                      delays=np.asarray(scan.delays, dtype=np.float64),
                      sos_true=sos_grid_truth(scan, ph), mask=free_node_mask(scan),
                      ip_true=render_ip(scan, blobs))


def random_sos(shape, v0: float, rng: np.random.Generator, amp: float = 0.04, smooth: int = 2) -> np.ndarray:
    """A smooth random SOS field around v0 (box-filtered noise), for parity tests."""
    z = rng.normal(size=shape)
    for _ in range(smooth):
        z = (z + np.roll(z, 1, 0) + np.roll(z, -1, 0) + np.roll(z, 1, 1) + np.roll(z, -1, 1)) / 5.0
    z = z / (np.abs(z).max() + 1e-30)
    return v0 + amp * z


def random_spectra(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian test data."""
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


__all__ = ["Scan", "TINY", "PAPER", "WORKLOADS", "describe", "uniform_delays", "delays_from_sos_offsets",
           "SosPhantom", "Blobs", "make_sos_phantom", "make_blobs", "render_ip", "sos_grid_truth",
           "free_node_mask", "axis", "channel_data", "travel_times", "point_source_data", "ScanInputs",
           "make_inputs", "random_sos", "random_spectra"]
