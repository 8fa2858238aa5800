"""Seeded synthetic inputs shared by the GPU library's tests and benches and
by the CPU oracle. Problem descriptions only: no transport arithmetic."""
from .problems import *  # noqa: F401,F403
