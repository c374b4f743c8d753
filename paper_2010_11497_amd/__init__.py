"""Cluster-and-Conquer (C^2) KNN-graph construction for AMD MI355X (gfx950)."""
