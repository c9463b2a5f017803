"""Writes the predictor's parameters as the C include compiled into the
library (paper_1809_04384_amd/csrc/rank_mlp_weights.inc): feature mean and
deviation, weight matrices rounded to BF16 (round to nearest even, stored as
the upper 16 bits of the float), FP32 biases."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
INC = os.path.join(HERE, "..", "csrc", "rank_mlp_weights.inc")
NF, NH = 12, 128


def bf16_bits(a):
    """float32 -> bfloat16 bits, round to nearest even."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return r.astype(np.uint16)


def bf16_round(a):
    """The float32 values the BF16 weights represent."""
    return (bf16_bits(a).astype(np.uint32) << 16).view(np.float32)


def write_inc(p, path=INC, note=""):
    """p: dict with mean, std [12], W1 [128, 12], b1, W2 [128, 128], b2, W3, b3, W4 [128], b4."""
    def arr(name, qual, ctype, vals, fmt):
        body = ", ".join(fmt(v) for v in np.ravel(vals))
        return "%s %s %s[%d] = {%s};\n" % (qual, ctype, name, np.size(vals), body)
    f32 = lambda v: "%.9ef" % float(v)
    hexb = lambda v: "0x%04x" % int(v)
    out = ["// Parameters of the learned rank predictor, written by\n",
           "// paper_1809_04384_amd/rank_model/weights.py%s.\n" % ((" (" + note + ")") if note else ""),
           arr("kMlpMean", "__constant__", "float", p["mean"], f32),
           arr("kMlpStd", "__constant__", "float", p["std"], f32),
           arr("kMlpW1", "__device__ const", "uint16_t", bf16_bits(p["W1"]), hexb),
           arr("kMlpB1", "__device__ const", "float", p["b1"], f32),
           arr("kMlpW2", "__device__ const", "uint16_t", bf16_bits(p["W2"]), hexb),
           arr("kMlpB2", "__device__ const", "float", p["b2"], f32),
           arr("kMlpW3", "__device__ const", "uint16_t", bf16_bits(p["W3"]), hexb),
           arr("kMlpB3", "__device__ const", "float", p["b3"], f32),
           arr("kMlpW4", "__device__ const", "uint16_t", bf16_bits(p["W4"]), hexb),
           "constexpr float kMlpB4 = %s;\n" % f32(p["b4"])]
    with open(path, "w") as fh:
        fh.write("".join(out))


def placeholder():
    """Parameters that predict rank 16 everywhere (before training)."""
    return {"mean": np.zeros(NF), "std": np.ones(NF), "W1": np.zeros((NH, NF)), "b1": np.zeros(NH),
            "W2": np.zeros((NH, NH)), "b2": np.zeros(NH), "W3": np.zeros((NH, NH)), "b3": np.zeros(NH),
            "W4": np.zeros(NH), "b4": np.log2(17.0)}


if __name__ == "__main__":
    write_inc(placeholder(), note="placeholder")
