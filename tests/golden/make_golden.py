"""Write the closed-form fixtures under tests/golden/ (calls only oracle/).

box_room_image_paths.txt: every reflection sequence with at most two
reflections that the image method realises in the empty 10 x 8 x 3 m room
with TX (2, 2, 1.5) and RX (7, 5, 1.5), with its exact squared length.
Face ids: 0 floor, 1 ceiling, 2 wall x=0, 3 wall x=10, 4 wall y=0, 5 wall y=8.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import image_method  # noqa: E402


def main():
    paths = image_method.box_room_paths((2.0, 2.0, 1.5), (7.0, 5.0, 1.5), (10.0, 8.0, 3.0), 2)
    lines = ["# image-method paths, empty box room 10x8x3, TX (2,2,1.5), RX (7,5,1.5), <= 2 reflections",
             "# columns: sequence (face ids, '-' for line of sight)  squared length (m^2)"]
    for seq in sorted(paths, key=lambda s: (len(s), s)):
        L = paths[seq][0]
        name = "-" if not seq else ",".join(str(x) for x in seq)
        lines.append(f"{name} {round(L * L, 6):.6f}")
    with open(os.path.join(HERE, "box_room_image_paths.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
