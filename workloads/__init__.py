"""Seeded synthetic inputs shared by the tests and the benchmark (no codec logic)."""
from .mixes import (MIXES, SCRIPT_MIXES, SEED_BATCH, SEED_MIX1M, SEED_SERVE, SEED_UTF8,
                    SEED_UTF8_INVALID, SEED_UTF16, SEED_UTF16_INVALID, StringBatch, TextBuffer,
                    draw_codepoints, lognormal_lengths, make_batch, make_buffer, make_requests, random_text,
                    RequestSet)
