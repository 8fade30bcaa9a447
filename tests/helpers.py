"""Shared test helpers: conversion of generated problems to oracle costs, error metrics."""
from __future__ import annotations

import numpy as np

import oracle


def oracle_cost(pr) -> "oracle.Cost":
    """Oracle cost built from the same float32 inputs the GPU sees (upcast to float64)."""
    if pr.C is not None:
        return oracle.Cost(C=pr.C.astype(np.float64))
    return oracle.Cost(x=pr.x.astype(np.float64), y=pr.y.astype(np.float64), p=pr.p)


def rel_inf(a, b) -> float:
    """||a - b||_inf / ||b||_inf (vector relative error)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = float(np.max(np.abs(b))) if b.size else 1.0
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)
