"""Placeholder; replaced by the binding below."""
