"""Seeded synthetic inputs (detector geometry, module map, events, model weights)."""
