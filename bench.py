"""placeholder; replaced below"""
DEFAULT_P = 64
DEFAULT_DEPTH = 1
